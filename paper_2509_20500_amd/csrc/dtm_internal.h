// Internal types shared by the host library and the kernels.  Plain C++,
// no HIP dependency, so the host-only translation unit builds with g++.
#pragma once

#include <cstddef>
#include <cstdint>

#include "dtm.h"

// Tuning constants (compile time).
#ifndef DTM_POOL_PAD
#define DTM_POOL_PAD 0  // bytes added between consecutive matrices in the pool
#endif
#ifndef DTM_NT_LOADS
#define DTM_NT_LOADS 1  // stream matrix reads with non-temporal loads
#endif

namespace dtm {

// Per-pixel metadata resident in device memory (batched path).  Offsets are
// in elements of the plan's dtype.
struct PixelMeta {
  double t_r;     // period
  double tau;     // pulse centre
  double sigma;   // pulse width
  double S;       // signal photons / period
  double B;       // background photons / period
  int32_t n;      // bins
  int32_t l;      // dead-time shift in bins (Theorem 2)
  int32_t ld;     // row stride of the pixel's matrix (n rounded up to 16 bytes)
  int32_t index;  // position of the pixel in the caller's arrays
  int64_t pi_off;   // offset of pi / x0 in the packed vectors (sum of n)
  int64_t vec_off;  // offset of per-pixel vectors in the workspace (sum of ld)
  int64_t mat_off;  // offset of the pixel's matrix in the matrix pool (sum of n*ld)
  int64_t out_off;  // offset of the pixel's matrix in a caller's packed output (sum of n*n)
  int64_t part_off; // banded pixels: offset (in doubles) of the band partial sums
  int32_t bands;    // banded pixels: row bands (0 for pixels of the fused kernel)
  int32_t big;      // position in the banded-pixel list, or -1
  double t_d;       // dead time (Monte Carlo simulator)
  double e_s, e_b;  // exp(-S), exp(-B), from the host's libm (Monte Carlo simulator)
  double frac;      // interpolated shift: weight f of base row i + l + 1 (0 otherwise)
  int32_t lam_mode; // 0: lambda at the bin centre, 1: bin-mean lambda, 2: bin integral
  int32_t pad2;
};
static_assert(sizeof(PixelMeta) == 144, "PixelMeta layout");

// One work item of the banded sweep: a band of rows times a block of columns
// of one pixel.
struct BandItem {
  int32_t meta;      // index into the plan's PixelMeta array
  int32_t band;      // row band
  int32_t colblock;  // column block
  int32_t pad;
};

// Solver options as the kernels see them.
struct KOpts {
  double tol;
  double safety;
  int32_t max_iter;
  int32_t stop_rule;
  int32_t final_check;
  int32_t pad;    // host only: 1 = the plan has no dense matrix pool
  int32_t model;  // host only: DTM_FLAG_SHIFT_* / LAMBDA_BIN_MEAN / BIN_INTEGRAL
  int32_t start_flux;  // batched dense solver: start from lambda / sum(lambda)
};

// Convergence bookkeeping of one pixel, shared by both solvers.
struct StopState {
  double c1, c2, c3;  // last three L1 changes (c1 newest)
  double rho;         // |lambda_2| estimate
  double gain;        // estimated error of the iterate per unit of change
  double contr;       // estimated contraction of the change per sweep
  double resid;       // float64 residual of the last check sweep
  double dd_prev;     // ||d_{t-1}||_2^2 of the previous difference vector
  int32_t iter;       // sweeps since the (re)start
  int32_t total_iter; // all sweeps
  int32_t check_next; // next sweep is the float64 check
  int32_t done;
  int32_t status;     // DTM_OK / DTM_ENOTCONV
  int32_t flags;      // DTM_INFO_*
  int32_t warm;       // started from a caller's vector
  int32_t stalled;    // changes stopped decreasing at the precision floor
};

// Per-pixel iteration state of the single-pixel (multi-launch) solver.
struct SolveState {
  StopState s;
  double sum_y;  // sum of the last product (diagnostic)
  double pad;
};

// Shared host logic (dtm_host.cpp).
int validate_scene(const dtm_scene& s, dtm_dtype dt, int32_t lam_mode = 0);
bool degenerate_scene(const dtm_scene& s, dtm_dtype dt, int32_t lam_mode);
int shift_bins(const dtm_scene& s, int32_t* l);
void model_shift(const dtm_scene& s, int32_t model, int32_t* l, double* frac);
int32_t model_lam_mode(int32_t model);
int fill_opts(const dtm_solve_opts* opt, KOpts* k, int32_t* check_every);
// Float64 continuation of the pixels of a bound plan still running after
// their dense sweeps: the one-block pixels (banded = 0) or the banded ones
// (banded = 1) (dtm_factored.hip; launch only, on the hipStream_t stream).
int launch_dense_tail(const dtm_plan* plan, int banded, void* pi, dtm_solve_info* infos, void* stream);
constexpr int32_t padded_ld(int32_t n, dtm_dtype dt) {
  const int32_t vec = dt == DTM_F32 ? 4 : 2;  // 16 bytes
  return (n + vec - 1) / vec * vec;
}
constexpr size_t dtype_size(dtm_dtype dt) { return dt == DTM_F32 ? 4 : 8; }
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace layout of the single-pixel entry points (byte offsets).  The
// band count caps the float64 partial sums at 256 rows of length ld; y and
// the per-block sums (sum y, sum |y - x|) serve the two-stage combine.
struct SingleLayout {
  int32_t ld, bands, band_rows, cblocks;
  size_t off_colf, off_invs, off_x, off_scal, off_state, off_dprev, off_part, off_y, off_bsum, total;
};
constexpr SingleLayout single_layout(int32_t n, dtm_dtype dt) {
  SingleLayout L{};
  L.ld = padded_ld(n, dt);
  // bands of about 32 rows up to 2048 bins (a 1000-bin matrix is swept by 64
  // workgroups), of about 64 rows above
  const int32_t want = n <= 2048 ? (n + 31) / 32 : (n + 63) / 64;
  L.bands = want < 256 ? want : 256;
  L.band_rows = (n + L.bands - 1) / L.bands;
  L.bands = (n + L.band_rows - 1) / L.band_rows;
  const size_t es = dtype_size(dt);
  size_t off = 0;
  L.off_colf = off; off = align256(off + es * L.ld);
  L.off_invs = off; off = align256(off + es * L.ld);
  L.off_x = off;    off = align256(off + es * L.ld);
  L.off_scal = off; off = align256(off + 64);
  L.off_state = off; off = align256(off + sizeof(SolveState));
  L.off_dprev = off; off = align256(off + 8 * static_cast<size_t>(L.ld));
  L.off_part = off; off = align256(off + 8 * static_cast<size_t>(L.bands) * L.ld);
  L.cblocks = (n + 255) / 256;
  L.off_y = off;    off = align256(off + 8 * static_cast<size_t>(L.ld));
  L.off_bsum = off; off = align256(off + 16 * static_cast<size_t>(L.cblocks));
  L.total = off;
  return L;
}

}  // namespace dtm

#include <vector>

// The host side of a batched plan.  Pixels are stored in launch order
// (descending n, so the largest pixels start first); meta[i].index maps back
// to the caller's order.
struct dtm_plan {
  dtm_dtype dt;
  dtm::KOpts kopts;
  int32_t check_every;
  dtm_tile_config tiles;
  std::vector<dtm::PixelMeta> meta;
  int32_t n_pixels;
  int32_t max_n;
  int32_t max_ld;
  int64_t pi_elems;    // sum n
  int64_t mat_elems;   // sum n*n
  int64_t pool_elems;  // sum n*ld
  int64_t vec_elems;   // sum ld
  // pixels of the fused one-block kernel and of the banded multi-block path
  std::vector<int32_t> small_sel, big_sel;
  std::vector<dtm::BandItem> items;
  // the building sweep's items when band_cpt > 1: the same bands in column
  // blocks of one vector per thread (256 x 4 float / 2 double columns), so
  // that the matrix writes are spread over four or two times as many
  // workgroups; the partial sums they write are the same
  std::vector<dtm::BandItem> build_items;
  // banded combine, stage 1: one item per column block of each banded pixel
  // (band 0), and each banded pixel's first column block in that list
  std::vector<dtm::BandItem> citems;
  std::vector<int32_t> cbase;
  int32_t max_n_small, max_ld_small, max_n_big, max_ld_big;
  int32_t band_threads, band_cpt;  // banded sweep block size and column chunks per thread
  int64_t part_elems;              // doubles of band partial sums
  // workspace layout, byte offsets
  size_t off_meta, off_pool, off_colf, off_invs, off_scal, off_state, total_bytes;
  size_t off_small, off_big, off_items, off_xbuf, off_dprev, off_part, off_fact;
  size_t off_citems, off_cbase, off_bsum, off_ybuf, off_queue;
  size_t off_live;     // banded path: int32 per launched sweep, the work items still running after it
  size_t off_build_items;
  void* ws;            // bound workspace (device), or nullptr
  size_t ws_bytes;
  // created at bind: a second stream (default priority) and two events that
  // fork the fused kernel off the caller's stream and join it back
  void* aux_stream;
  void* ev_fork;
  void* ev_join;
};
