// Host-only logic of the library: argument validation, the dead-time shift
// rule, solver options and batched plans.  No HIP calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "dtm_internal.h"

namespace dtm {

// Normal tail beyond z on z's side, and the normal mass on [za, zb] from the
// tails at its ends, each difference taken where it keeps its digits.
static double host_tail(double z) { return 0.5 * std::erfc(std::fabs(z) * 0.70710678118654752440); }
static double host_mass(double za, double zb) {
  const double ta = host_tail(za), tb = host_tail(zb);
  if (za >= 0.0) return ta - tb;
  if (zb <= 0.0) return tb - ta;
  return 1.0 - ta - tb;
}

// g_j = lambda_j exp(-F_j) of bin j (the column factor of every row of the
// base matrix, Section 3.4) evaluated on the host in float64, under the
// flux sampling of lam_mode (0: lambda at the centre; 1: lambda averaged
// over the bin; 2: lambda e^{-F} averaged over the bin).  F is Theorem 1's
// cumulative flux with the pulse cut to [0, t_r).
static double host_g(const dtm_scene& s, int32_t j, int32_t lam_mode) {
  const double delta = s.period_ns / s.n_bins, is = 1.0 / s.pulse_sigma_ns;
  const double lo = j * delta, mid = lo + 0.5 * delta, hi = lo + delta;
  const double z0 = -s.pulse_center_ns * is;
  const auto F = [&](double t) {
    return s.signal_flux * host_mass(z0, (t - s.pulse_center_ns) * is) + s.background_flux * t / s.period_ns;
  };
  const double Fm = F(mid);
  if (lam_mode == 0) {
    const double z = (mid - s.pulse_center_ns) * is;
    const double lam = s.signal_flux * std::exp(-0.5 * z * z) * (0.39894228040143267794 * is) +
                       s.background_flux / s.period_ns;
    return lam * std::exp(-Fm);
  }
  const double dF = s.signal_flux * host_mass((lo - s.pulse_center_ns) * is, (hi - s.pulse_center_ns) * is) +
                    s.background_flux * delta / s.period_ns;
  if (lam_mode == 1) return dF / delta * std::exp(-Fm);
  return std::exp(-F(lo)) * -std::expm1(-dF) / delta;
}

// Scene validation (Section 2.2's theta; flux model of Eq. arrival_flux).
// float32 needs exp(-Lambda) and exp(-F) to stay normal: S + B <= 80.
// A scene whose flux underflows at every bin leaves every row of the matrix
// zero (the chain is undefined): g_j is largest at the first bin (the
// background term, where F is smallest) or at a bin next to the pulse
// centre, so those bins decide; below the smallest normal number of the
// dtype the scene is rejected.
int validate_scene(const dtm_scene& s, dtm_dtype dt, int32_t lam_mode) {
  const double v[6] = {s.period_ns, s.dead_time_ns, s.pulse_center_ns,
                       s.pulse_sigma_ns, s.signal_flux, s.background_flux};
  for (double x : v)
    if (!std::isfinite(x)) return DTM_EINVAL;
  if (s.period_ns <= 0.0 || s.dead_time_ns < 0.0 || s.pulse_sigma_ns <= 0.0) return DTM_EINVAL;
  if (s.signal_flux < 0.0 || s.background_flux < 0.0) return DTM_EINVAL;
  if (!(s.signal_flux + s.background_flux > 0.0)) return DTM_EINVAL;
  if (s.n_bins < 2 || s.n_bins > DTM_MAX_BINS || s.reserved != 0) return DTM_EINVAL;
  if (dt != DTM_F32 && dt != DTM_F64) return DTM_EINVAL;
  const double lim = dt == DTM_F32 ? 80.0 : 700.0;
  if (s.signal_flux + s.background_flux > lim) return DTM_ENOTSUP;
  if (degenerate_scene(s, dt, lam_mode)) return DTM_EINVAL;
  return DTM_OK;
}

bool degenerate_scene(const dtm_scene& s, dtm_dtype dt, int32_t lam_mode) {
  const double tiny = dt == DTM_F32 ? 1.17549435082228750797e-38 : 2.22507385850720138309e-308;
  // the background alone keeps every g_j >= (B / t_r) exp(-Lambda), Lambda <= S + B
  if (s.background_flux / s.period_ns * std::exp(-(s.signal_flux + s.background_flux)) >= tiny) return false;
  const double delta = s.period_ns / s.n_bins;
  const double jt = std::floor(s.pulse_center_ns / delta);
  const int32_t jc = static_cast<int32_t>(std::min<double>(std::max<double>(jt, 0.0), s.n_bins - 1));
  double gmax = host_g(s, 0, lam_mode);
  for (int32_t j = std::max(jc - 1, 0); j <= std::min(jc + 1, s.n_bins - 1); ++j)
    gmax = std::max(gmax, host_g(s, j, lam_mode));
  return !(gmax >= tiny);
}

// l = ceil(x_d / Delta) mod n_b (Theorem 2) with x_d = t_d mod t_r.
// q = x_d * n_b / t_r; a q within 1e-9 (relative) of an integer is that
// integer: the dead time is a whole number of bins and the shifted centre is
// itself a centre, so there is nothing to round up.
int shift_bins(const dtm_scene& s, int32_t* l) {
  const double x_d = std::fmod(s.dead_time_ns, s.period_ns);
  const double q = x_d * static_cast<double>(s.n_bins) / s.period_ns;
  const double r = std::nearbyint(q);
  double lq;
  if (std::fabs(q - r) <= 1e-9 * std::max(1.0, q))
    lq = r;
  else
    lq = std::ceil(q);
  int64_t li = static_cast<int64_t>(lq) % s.n_bins;
  if (li < 0) li += s.n_bins;
  *l = static_cast<int32_t>(li);
  return DTM_OK;
}

// Shift of a pixel under the discretisation flags.  SHIFT_NEAREST: the bin
// of the shifted centre, (i + 1/2 + q) Delta in (j Delta, (j + 1) Delta],
// i.e. row i + ceil(q - 1/2); SHIFT_INTERP: q = l + frac with 0 <= frac < 1.
// Both snap to an integer within 1e-9 (relative), like Theorem 2's shift.
void model_shift(const dtm_scene& s, int32_t model, int32_t* l, double* frac) {
  *frac = 0.0;
  if (!(model & (DTM_FLAG_SHIFT_NEAREST | DTM_FLAG_SHIFT_INTERP))) {
    shift_bins(s, l);
    return;
  }
  const double x_d = std::fmod(s.dead_time_ns, s.period_ns);
  const double q = x_d * static_cast<double>(s.n_bins) / s.period_ns;
  const double p = (model & DTM_FLAG_SHIFT_NEAREST) ? q - 0.5 : q;
  const double r = std::nearbyint(p);
  double lq;
  if (std::fabs(p - r) <= 1e-9 * std::max(1.0, std::fabs(p))) {
    lq = r;
  } else if (model & DTM_FLAG_SHIFT_NEAREST) {
    lq = std::ceil(p);
  } else {
    lq = std::floor(p);
    *frac = p - lq;
  }
  int64_t li = static_cast<int64_t>(lq) % s.n_bins;
  if (li < 0) li += s.n_bins;
  *l = static_cast<int32_t>(li);
}

int32_t model_lam_mode(int32_t model) {
  if (model & DTM_FLAG_LAMBDA_BIN_MEAN) return 1;
  if (model & DTM_FLAG_BIN_INTEGRAL) return 2;
  return 0;
}

int fill_opts(const dtm_solve_opts* opt, KOpts* k, int32_t* check_every) {
  dtm_solve_opts o;
  if (opt) {
    o = *opt;
  } else {
    o.tol_l1 = 1e-6;
    o.safety = 0.25;
    o.max_iter = 1000;
    o.check_every = 4;
    o.stop_rule = DTM_STOP_BOUND;
    o.flags = 0;
  }
  if (!(o.tol_l1 > 0.0) || !std::isfinite(o.tol_l1)) return DTM_EINVAL;
  if (!(o.safety > 0.0 && o.safety <= 1.0)) return DTM_EINVAL;
  if (o.max_iter < 1 || o.check_every < 1) return DTM_EINVAL;
  if (o.stop_rule != DTM_STOP_CHANGE && o.stop_rule != DTM_STOP_BOUND) return DTM_EINVAL;
  constexpr int32_t kModel =
      DTM_FLAG_SHIFT_NEAREST | DTM_FLAG_SHIFT_INTERP | DTM_FLAG_LAMBDA_BIN_MEAN | DTM_FLAG_BIN_INTEGRAL;
  if (o.flags & ~(DTM_FLAG_NO_FINAL_CHECK | DTM_FLAG_NO_DENSE | DTM_FLAG_START_FLUX | kModel)) return DTM_EINVAL;
  if ((o.flags & DTM_FLAG_SHIFT_NEAREST) && (o.flags & DTM_FLAG_SHIFT_INTERP)) return DTM_EINVAL;
  if ((o.flags & DTM_FLAG_LAMBDA_BIN_MEAN) && (o.flags & DTM_FLAG_BIN_INTEGRAL)) return DTM_EINVAL;
  k->tol = o.tol_l1;
  k->safety = o.safety;
  k->max_iter = o.max_iter;
  k->stop_rule = o.stop_rule;
  k->final_check = (o.flags & DTM_FLAG_NO_FINAL_CHECK) ? 0 : 1;
  k->pad = (o.flags & DTM_FLAG_NO_DENSE) ? 1 : 0;  // no dense pool
  k->model = o.flags & kModel;
  k->start_flux = (o.flags & DTM_FLAG_START_FLUX) ? 1 : 0;
  if (check_every) *check_every = o.check_every;
  return DTM_OK;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace dtm

using namespace dtm;

extern "C" {

const char* dtm_status_string(int status) {
  switch (status) {
    case DTM_OK: return "ok";
    case DTM_EINVAL: return "invalid argument";
    case DTM_ENOTCONV: return "power iteration did not converge within max_iter";
    case DTM_EHIP: return "HIP runtime error";
    case DTM_EALIAS: return "input and output buffers overlap";
    case DTM_ENOSPACE: return "workspace too small";
    case DTM_ENOTSUP: return "not supported by the library";
    default: return "unknown status";
  }
}

int dtm_version(void) { return 10000; }

int dtm_validate_scene(const dtm_scene* s) {
  if (!s) return DTM_EINVAL;
  return validate_scene(*s, DTM_F64);
}

int dtm_shift_bins(const dtm_scene* s, int32_t* l_out) {
  if (!s || !l_out) return DTM_EINVAL;
  const int st = validate_scene(*s, DTM_F64);
  if (st != DTM_OK) return st;
  return shift_bins(*s, l_out);
}

int dtm_model_shift(const dtm_scene* s, int32_t flags, int32_t* l_out, double* frac_out) {
  if (!s || !l_out || !frac_out) return DTM_EINVAL;
  if ((flags & DTM_FLAG_SHIFT_NEAREST) && (flags & DTM_FLAG_SHIFT_INTERP)) return DTM_EINVAL;
  const int st = validate_scene(*s, DTM_F64);
  if (st != DTM_OK) return st;
  model_shift(*s, flags, l_out, frac_out);
  return DTM_OK;
}

size_t dtm_workspace_bytes(int32_t n, dtm_dtype dt) {
  if (n < 2 || n > DTM_MAX_BINS || (dt != DTM_F32 && dt != DTM_F64)) return 0;
  return single_layout(n, dt).total;
}

int dtm_plan_create(const dtm_scene* scenes_host, int32_t n_pixels, dtm_dtype dt,
                    const dtm_solve_opts* opt, const dtm_tile_config* tiles,
                    dtm_plan** plan_out) {
  if (!plan_out) return DTM_EINVAL;
  *plan_out = nullptr;
  if (!scenes_host || n_pixels < 1) return DTM_EINVAL;
  if (dt != DTM_F32 && dt != DTM_F64) return DTM_EINVAL;
  KOpts ko;
  int32_t ce = 4;
  int st = fill_opts(opt, &ko, &ce);
  if (st != DTM_OK) return st;
  // the dense kernels take whole rows of the shifted matrix
  if ((ko.model & DTM_FLAG_SHIFT_INTERP) && !ko.pad) return DTM_ENOTSUP;
  for (int32_t p = 0; p < n_pixels; ++p) {
    st = validate_scene(scenes_host[p], dt, model_lam_mode(ko.model));
    if (st != DTM_OK) return st;
  }
  dtm_plan* plan = new (std::nothrow) dtm_plan();
  if (!plan) return DTM_EINVAL;
  plan->dt = dt;
  plan->kopts = ko;
  plan->check_every = ce;
  static_assert(sizeof(dtm_tile_config) == 36, "dtm_tile_config layout");
  dtm_tile_config tc;
  std::memset(&tc, 0, sizeof(tc));
  if (tiles) tc = *tiles;
  const bool auto_threads = tc.fused_threads == 0;  // settled once the one-block pixels are known
  if (auto_threads) tc.fused_threads = 256;
  if (tc.fused_unroll == 0) tc.fused_unroll = 8;
  if (tc.fused_max_bins == 0) tc.fused_max_bins = 2048;
  if (tc.band_rows == 0) tc.band_rows = 1024;
  if (tc.dense_sweeps == 0) tc.dense_sweeps = std::min(ko.max_iter, 32);
  if (tc.band_cpt == 0) tc.band_cpt = 1;
  if ((tc.fused_threads != 256 && tc.fused_threads != 512) ||
      (tc.fused_unroll != 2 && tc.fused_unroll != 4 && tc.fused_unroll != 8) ||
      tc.fused_max_bins < 2 || tc.band_rows < 16 || tc.band_rows % 16 != 0 || tc.band_rows > 8192 ||
      tc.dense_sweeps < 1 || tc.dense_sweeps > ko.max_iter ||
      (tc.band_cpt != 1 && tc.band_cpt != 2 && tc.band_cpt != 4) ||
      (tc.independent_paths != 0 && tc.independent_paths != 1) || tc.fused_blocks < 0 ||
      tc.band_min_items < 0) {
    delete plan;
    return DTM_EINVAL;
  }
  // The fused kernel holds g, x and 1/S in LDS (3 ld elements) and at most 4
  // vectors of columns per thread of a 512-thread block.
  {
    const int32_t vn = dt == DTM_F32 ? 4 : 2;
    const int32_t cap_regs = 512 * vn * 4;
    const int32_t cap_lds = static_cast<int32_t>((150 * 1024) / (3 * dtype_size(dt)));
    tc.fused_max_bins = std::min(tc.fused_max_bins, std::min(cap_regs, cap_lds));
  }
  plan->tiles = tc;
  plan->n_pixels = n_pixels;

  // Launch order: longest expected job first, so that the last blocks to
  // start are short ones.  A pixel's cost is n^2 bytes per sweep times its
  // sweep count; the sweep count grows as the spectral gap 1 - |lambda_2|
  // shrinks, which happens as the background flux B grows (Section 4), so
  // the expected cost is taken as n^2 (1 + 2 B).  Stable on input index.
  std::vector<int32_t> order(n_pixels);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> cost(n_pixels);
  for (int32_t p = 0; p < n_pixels; ++p) {
    const double nn = static_cast<double>(scenes_host[p].n_bins);
    cost[p] = nn * nn * (1.0 + 2.0 * scenes_host[p].background_flux);
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
  // Offsets in the caller's order.
  std::vector<int64_t> pi_off(n_pixels), out_off(n_pixels);
  int64_t acc_pi = 0, acc_out = 0;
  for (int32_t p = 0; p < n_pixels; ++p) {
    pi_off[p] = acc_pi;
    out_off[p] = acc_out;
    acc_pi += scenes_host[p].n_bins;
    acc_out += static_cast<int64_t>(scenes_host[p].n_bins) * scenes_host[p].n_bins;
  }
  plan->pi_elems = acc_pi;
  plan->mat_elems = acc_out;
  plan->meta.resize(n_pixels);
  int64_t acc_vec = 0, acc_pool = 0;
  int32_t max_n = 0, max_ld = 0;
  static_assert(DTM_POOL_PAD % 16 == 0, "pool stagger must keep 16-byte alignment");
  for (int32_t q = 0; q < n_pixels; ++q) {
    const int32_t p = order[q];
    const dtm_scene& s = scenes_host[p];
    PixelMeta& m = plan->meta[q];
    m.t_r = s.period_ns;
    m.tau = s.pulse_center_ns;
    m.sigma = s.pulse_sigma_ns;
    m.S = s.signal_flux;
    m.B = s.background_flux;
    m.n = s.n_bins;
    model_shift(s, ko.model, &m.l, &m.frac);
    m.lam_mode = model_lam_mode(ko.model);
    m.pad2 = 0;
    m.ld = padded_ld(s.n_bins, dt);
    m.index = p;
    m.t_d = s.dead_time_ns;
    m.e_s = std::exp(-s.signal_flux);
    m.e_b = std::exp(-s.background_flux);
    m.pi_off = pi_off[p];
    m.vec_off = acc_vec;
    m.mat_off = acc_pool;
    m.out_off = out_off[p];
    acc_vec += m.ld;
    // Consecutive matrices are staggered by DTM_POOL_PAD bytes so that the
    // many blocks streaming their own matrix in step do not start on the
    // same HBM channel.
    acc_pool += static_cast<int64_t>(m.n) * m.ld +
                static_cast<int64_t>(DTM_POOL_PAD) / static_cast<int64_t>(dtype_size(dt));
    max_n = std::max(max_n, m.n);
    max_ld = std::max(max_ld, m.ld);
  }
  plan->vec_elems = acc_vec;
  plan->pool_elems = acc_pool;
  plan->max_n = max_n;
  plan->max_ld = max_ld;

  // Split: pixels up to fused_max_bins take the one-block fused kernel, the
  // others the banded path (row bands x column blocks, one block each).
  const int32_t vn = dt == DTM_F32 ? 4 : 2;
  plan->band_threads = 256;
  plan->band_cpt = tc.band_cpt;
  const int32_t colw = plan->band_threads * vn * plan->band_cpt;
  plan->max_n_small = plan->max_ld_small = plan->max_n_big = plan->max_ld_big = 0;
  int64_t acc_part = 0;
  for (int32_t q = 0; q < n_pixels; ++q) {
    PixelMeta& m = plan->meta[q];
    if (m.n <= tc.fused_max_bins) {
      m.bands = 0;
      m.big = -1;
      m.part_off = 0;
      plan->small_sel.push_back(q);
      plan->max_n_small = std::max(plan->max_n_small, m.n);
      plan->max_ld_small = std::max(plan->max_ld_small, m.ld);
    } else {
      m.bands = (m.n + tc.band_rows - 1) / tc.band_rows;
      m.big = static_cast<int32_t>(plan->big_sel.size());
      m.part_off = acc_part;
      acc_part += static_cast<int64_t>(m.bands) * m.ld;
      plan->big_sel.push_back(q);
      plan->max_n_big = std::max(plan->max_n_big, m.n);
      plan->max_ld_big = std::max(plan->max_ld_big, m.ld);
      const int32_t cblocks = (m.n + colw - 1) / colw;
      for (int32_t b = 0; b < m.bands; ++b)
        for (int32_t cb = 0; cb < cblocks; ++cb) plan->items.push_back(BandItem{q, b, cb, 0});
      if (plan->band_cpt > 1) {
        const int32_t colw1 = plan->band_threads * vn;
        const int32_t cblocks1 = (m.n + colw1 - 1) / colw1;
        for (int32_t b = 0; b < m.bands; ++b)
          for (int32_t cb = 0; cb < cblocks1; ++cb) plan->build_items.push_back(BandItem{q, b, cb, 0});
      }
      // the combine's column blocks (stage 1) and where the pixel's start
      plan->cbase.push_back(static_cast<int32_t>(plan->citems.size()));
      for (int32_t cb = 0; cb < cblocks; ++cb) plan->citems.push_back(BandItem{q, 0, cb, 0});
    }
  }
  plan->part_elems = acc_part;
  // A one-block pixel is streamed by one workgroup, whose rate is bounded by
  // the bytes its threads keep in flight: pixels above 1024 bins get twice
  // the threads by default.
  if (auto_threads && plan->max_n_small > 1024) plan->tiles.fused_threads = 512;
  const size_t es = dtype_size(dt);
  size_t off = 0;
  plan->off_meta = off;
  off = align_up(off + sizeof(PixelMeta) * n_pixels, 256);
  plan->off_colf = off;
  off = align_up(off + es * acc_vec, 256);
  plan->off_invs = off;
  off = align_up(off + es * acc_vec, 256);
  plan->off_scal = off;
  off = align_up(off + 8 * static_cast<size_t>(n_pixels), 256);
  plan->off_state = off;
  off = align_up(off + sizeof(SolveState) * n_pixels, 256);
  plan->off_small = off;
  off = align_up(off + sizeof(int32_t) * (plan->small_sel.size() + 1), 256);
  plan->off_big = off;
  off = align_up(off + sizeof(int32_t) * (plan->big_sel.size() + 1), 256);
  plan->off_items = off;
  off = align_up(off + sizeof(BandItem) * (plan->items.size() + 1), 256);
  plan->off_queue = off;
  off = align_up(off + 256, 256);
  plan->off_live = off;
  off = align_up(off + sizeof(int32_t) * (static_cast<size_t>(plan->tiles.dense_sweeps) + 1), 256);
  plan->off_build_items = off;
  off = align_up(off + sizeof(BandItem) * (plan->build_items.size() + 1), 256);
  plan->off_citems = off;
  off = align_up(off + sizeof(BandItem) * (plan->citems.size() + 1), 256);
  plan->off_cbase = off;
  off = align_up(off + sizeof(int32_t) * (plan->cbase.size() + 1), 256);
  plan->off_bsum = off;
  off = align_up(off + 16 * (plan->citems.size() + 1), 256);
  plan->off_ybuf = off;
  off = align_up(off + 8 * acc_vec, 256);
  plan->off_xbuf = off;
  off = align_up(off + es * acc_vec, 256);
  plan->off_dprev = off;
  off = align_up(off + 8 * acc_vec, 256);
  plan->off_part = off;
  off = align_up(off + 8 * static_cast<size_t>(acc_part), 256);
  // float64 scratch of the factored solver and the spectral analysis:
  // g, 1/S, x, u, previous difference (5 vectors of ld per pixel)
  plan->off_fact = off;
  off = align_up(off + 5 * 8 * static_cast<size_t>(acc_vec), 256);
  plan->off_pool = off;
  if (!ko.pad) off = align_up(off + es * static_cast<size_t>(acc_pool), 256);
  plan->total_bytes = off;
  plan->ws = nullptr;
  plan->ws_bytes = 0;
  plan->aux_stream = plan->ev_fork = plan->ev_join = nullptr;
  *plan_out = plan;
  return DTM_OK;
}

size_t dtm_plan_workspace_bytes(const dtm_plan* plan) { return plan ? plan->total_bytes : 0; }
int64_t dtm_plan_pi_elems(const dtm_plan* plan) { return plan ? plan->pi_elems : -1; }
int64_t dtm_plan_matrix_elems(const dtm_plan* plan) { return plan ? plan->mat_elems : -1; }

int dtm_plan_offsets(const dtm_plan* plan, int64_t* pi_offsets, int64_t* mat_offsets) {
  if (!plan) return DTM_EINVAL;
  const int32_t n = plan->n_pixels;
  std::vector<int64_t> pi(n + 1), mat(n + 1);
  for (const PixelMeta& m : plan->meta) {
    pi[m.index] = m.pi_off;
    mat[m.index] = m.out_off;
  }
  pi[n] = plan->pi_elems;
  mat[n] = plan->mat_elems;
  if (pi_offsets) std::memcpy(pi_offsets, pi.data(), sizeof(int64_t) * (n + 1));
  if (mat_offsets) std::memcpy(mat_offsets, mat.data(), sizeof(int64_t) * (n + 1));
  return DTM_OK;
}

int dtm_plan_tiles(const dtm_plan* plan, dtm_tile_config* tiles_out) {
  if (!plan || !tiles_out) return DTM_EINVAL;
  *tiles_out = plan->tiles;
  return DTM_OK;
}

}  // extern "C"
