// Factored transition matrix: power iteration and spectral analysis in O(n)
// per matrix-vector product, without forming P~.
//
// Row i of the dead-time matrix (Section 3.4, Theorem 2) is
//   P~[i, j] = g_j w_kj / S_k,  k = (i + l) mod n,  g_j = lambda_j e^{-F_j},
//   w_kj = c = e^{-Lambda} for j < k and 1 otherwise,
// so with u_k = x_{(k - l) mod n} / S_k and U_j = sum_{k <= j} u_k,
//   (x P~)_j = g_j sum_k u_k w_kj = g_j (c U_{n-1} + (1 - c) U_j):
// one prefix scan per product.  Everything here is float64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "dtm_device.hpp"
#include "dtm_internal.h"

namespace dtm {
namespace fact {

constexpr int BT = 256;
constexpr int kLdsMaxN = 2048;  // largest n whose solver vectors are kept in LDS
constexpr int KSUB = 6;  // dimension of the subspace that the lambda_2 search iterates
// float64 vectors of ld per pixel in the spectral scratch: the solver's five
// (g, 1/S, pi, u, last difference), then the subspace basis Q and its image W
constexpr int NVEC = 5 + 2 * KSUB;
// of which the lambda_2 search keeps g, 1/S, pi and the basis and its image
// in LDS (n <= kSpecLdsMaxN)
constexpr int NVEC_LDS = 3 + 2 * KSUB;
constexpr int kSpecLdsMaxN = 1024;  // largest n whose spectral vectors are kept in LDS

// Chunk of bins owned by this thread (the layout of pixel_tables).
__device__ inline void chunk_of(int n, int& j0, int& j1) {
  const int ch = (n + BT - 1) / BT;
  j0 = min(static_cast<int>(threadIdx.x) * ch, n);
  j1 = min(j0 + ch, n);
}

// The vector the base rows see: x_{k - l}, or with an interpolated shift
// (row i = (1 - f) base row i + l + f base row i + l + 1)
// (1 - f) x_{k - l} + f x_{k - l - 1}; indices mod n.
template <typename X>
__device__ inline double shifted_x(X x, int n, int l, double f, int k) {
  int i = k - l;
  if (i < 0) i += n;
  if (f == 0.0) return x(i);
  const int i2 = i == 0 ? n - 1 : i - 1;
  return (1.0 - f) * x(i) + f * x(i2);
}

// y = x P~ (unnormalised).  u is scratch of n doubles; y may alias u but not
// x.  Ends with block barriers (inside the scan), so callers may reduce.
__device__ void apply(int n, int l, double f, const double* x, const double* g, const double* invs,
                      double c, double* u, double* y, double* red) {
  int j0, j1;
  chunk_of(n, j0, j1);
  double cs = 0.0;
  const auto xv = [x](int i) { return x[i]; };
  for (int k = j0; k < j1; ++k) {
    const double v = shifted_x(xv, n, l, f, k) * invs[k];
    u[k] = v;
    cs += v;
  }
  double tot;
  const double pre = block_exclusive_scan<BT>(cs, red, tot);
  double U = pre;
  for (int j = j0; j < j1; ++j) {
    U += u[j];
    y[j] = g[j] * (c * tot + (1.0 - c) * U);
  }
}

struct Vecs {
  double *g, *invs, *x, *u, *dp;
};

__device__ inline Vecs vecs(double* fact, int64_t vec_elems, const PixelMeta& m) {
  Vecs V;
  double* base = fact + m.vec_off;
  V.g = base;
  V.invs = base + vec_elems;
  V.x = base + 2 * vec_elems;
  V.u = base + 3 * vec_elems;
  V.dp = base + 4 * vec_elems;
  return V;
}

// Tables in float64 for one pixel; returns c = e^{-Lambda}.
__device__ double tables(const PixelMeta& m, const Vecs& V, double* red) {
  const double Lam = pixel_tables<double, BT>(m, V.g, nullptr, nullptr, red);
  const double c = exp(-Lam);
  row_normalisers<double, BT>(m.n, V.g, c, V.u, V.invs, red);
  __syncthreads();
  return c;
}

// Power iteration on the factored matrix from the iterate in V.x (every
// sweep float64, treated as a check sweep by the stop rule), continuing the
// stop state st.  Returns when st is done; V.x holds the result.
__device__ void power_loop(const PixelMeta& m, const Vecs& V, double c, KOpts o, StopState& st,
                           double* red) {
  const int n = m.n;
  int j0, j1;
  chunk_of(n, j0, j1);
  for (;;) {
    apply(n, m.l, m.frac, V.x, V.g, V.invs, c, V.u, V.u, red);
    double sy = 0.0, rs = 0.0;
    for (int j = j0; j < j1; ++j) {
      sy += V.u[j];
      rs += fabs(V.u[j] - V.x[j]);
    }
    block_sum2<BT>(sy, rs, red);  // every read of x by apply is done
    double ch = 0.0, dd = 0.0, ddp = 0.0;
    for (int j = j0; j < j1; ++j) {
      const double xn = V.u[j] / sy;
      const double d = xn - V.x[j];
      ch += fabs(d);
      dd += d * d;
      ddp += d * V.dp[j];
      V.dp[j] = d;
      V.x[j] = xn;
    }
    block_sum3<BT>(ch, dd, ddp, red);
    const bool restart = stop_update(st, o, ch, dd, ddp, rs, true, 1.1102230246251565e-16);
    if (restart) {
      for (int j = j0; j < j1; ++j) {
        V.x[j] = 1.0 / n;
        V.dp[j] = 0.0;
      }
    }
    __syncthreads();
    if (st.done) break;
  }
}

// Starting vector in V.x: x0 normalised to sum 1 when it is a positive
// finite vector, else uniform.  Returns whether x0 was taken.
template <typename TI>
__device__ bool power_start(const PixelMeta& m, const Vecs& V, const TI* x0, double* red) {
  const int n = m.n;
  int j0, j1;
  chunk_of(n, j0, j1);
  double sum = 0.0, bad = 0.0;
  if (x0) {
    for (int j = j0; j < j1; ++j) {
      const double v = static_cast<double>(x0[j]);
      if (!(v >= 0.0) || !isfinite(v)) bad += 1.0;
      else sum += v;
    }
  }
  block_sum2<BT>(sum, bad, red);
  const bool warm = x0 && bad == 0.0 && sum > 0.0 && isfinite(sum);
  for (int j = j0; j < j1; ++j) {
    V.x[j] = warm ? static_cast<double>(x0[j]) / sum : 1.0 / n;
    V.dp[j] = 0.0;
  }
  __syncthreads();
  return warm;
}

// Power iteration on the factored matrix from x0 (may be null: uniform).
// Returns the stop state; V.x holds the result.
template <typename TI>
__device__ StopState power(const PixelMeta& m, const Vecs& V, double c, const TI* x0, KOpts o,
                           double* red) {
  const bool warm = power_start(m, V, x0, red);
  StopState st;
  stop_init(st, warm ? 1 : 0, (x0 && !warm) ? DTM_INFO_WARM_REJECTED : 0);
  power_loop(m, V, c, o, st, red);
  return st;
}

// Pixels of the dense solver that used their dense sweeps (the tile's
// dense_sweeps) without stopping: the power iteration goes on from the pixel's current
// iterate with the factored product of the same matrix, every sweep in
// float64, until the stop rule ends it or max_iter sweeps since the start
// (or the warm start's restart) have been taken.  Pixels that stopped
// return at once.  The stop rule's contraction estimate starts afresh from
// the continued iterate.  Writes pi and the pixel's report, flagged
// DTM_INFO_CONTINUED.
template <typename T>
__global__ __launch_bounds__(BT) void k_dense_tail(const PixelMeta* __restrict__ metas,
                                                  const int32_t* __restrict__ sel,
                                                  double* __restrict__ fact, int64_t vec_elems,
                                                  const T* __restrict__ xbuf, SolveState* __restrict__ states,
                                                  T* __restrict__ pi_packed, dtm_solve_info* __restrict__ infos,
                                                  KOpts o) {
  __shared__ double red[3 * BT / kWave];
  const int q = sel[blockIdx.x];
  const PixelMeta m = metas[q];
  const StopState prev = states[q].s;
  if (prev.done) return;
  const Vecs V = vecs(fact, vec_elems, m);
  int j0, j1;
  chunk_of(m.n, j0, j1);
  StopState st = prev;
  if (prev.iter < o.max_iter) {
    const double c = tables(m, V, red);
    power_start(m, V, xbuf + m.vec_off, red);
    // the remaining sweeps of this start (the iterate is not re-run from
    // uniform when they run out, whatever the start was)
    stop_init(st, 0, 0);
    KOpts oc = o;
    oc.max_iter = o.max_iter - prev.iter;
    power_loop(m, V, c, oc, st, red);
    for (int j = j0; j < j1; ++j) pi_packed[m.pi_off + j] = static_cast<T>(V.x[j]);
    st.total_iter += prev.total_iter;
    st.flags |= prev.flags & (DTM_INFO_WARM_REJECTED | DTM_INFO_RESTARTED);
  } else {  // no sweeps left: the last iterate is the answer
    for (int j = j0; j < j1; ++j) pi_packed[m.pi_off + j] = xbuf[m.vec_off + j];
    st.done = 1;
    st.status = DTM_ENOTCONV;
  }
  st.flags |= DTM_INFO_CONTINUED;
  if (threadIdx.x == 0) {
    dtm_solve_info info = make_info(st);
    info.dense_sweeps = prev.total_iter;
    infos[m.index] = info;
    states[q].s = st;
  }
}

// k_dense_tail for pixels of at most 512 E bins, by 512 threads: thread t
// owns the ch = ceil(n / 512) bins from t ch on, and keeps their iterate,
// product and last difference in registers, and g and 1/S too for E <= 8
// (above, they are read from the workspace in every sweep: registers would
// spill); only the iterate also goes to LDS (one pad slot after every E bins, so the lanes' strided reads
// spread over the banks), for the shifted reads of the next product.  A sweep
// is one LDS pass, one block scan and two block sums, against six passes over
// global vectors in k_dense_tail.  Same steps, start and stop rule; sums in
// 8 waves instead of 4, so the last bits may differ.
constexpr int BTT = 512;

template <int E>
__device__ inline int tail_slot(int j) {
  return j + j / E;
}

template <int E>
constexpr size_t tail_lds_bytes() {
  return sizeof(double) * (static_cast<size_t>(BTT) * E + BTT);
}

template <typename T, int E>
__global__ __launch_bounds__(BTT) void k_dense_tail_reg(const PixelMeta* __restrict__ metas,
                                                        const int32_t* __restrict__ sel,
                                                        double* __restrict__ fact, int64_t vec_elems,
                                                        const T* __restrict__ xbuf,
                                                        SolveState* __restrict__ states,
                                                        T* __restrict__ pi_packed,
                                                        dtm_solve_info* __restrict__ infos, KOpts o) {
  __shared__ double red[3 * BTT / kWave];
  extern __shared__ double xs[];  // tail_lds_bytes<E>()
  const int q = sel[blockIdx.x];
  const PixelMeta m = metas[q];
  const StopState prev = states[q].s;
  if (prev.done) return;
  const int n = m.n;
  const int ch = (n + BTT - 1) / BTT;  // at most E (the launcher's choice of E)
  const int j0 = min(static_cast<int>(threadIdx.x) * ch, n);
  const int cnt = min(ch, n - j0);
  StopState st = prev;
  if (prev.iter >= o.max_iter) {  // no sweeps left: the last iterate is the answer
    for (int e = 0; e < cnt; ++e) pi_packed[m.pi_off + j0 + e] = xbuf[m.vec_off + j0 + e];
    st.done = 1;
    st.status = DTM_ENOTCONV;
  } else {
    const Vecs V = vecs(fact, vec_elems, m);
    // tables in the chunks of this block's 512 threads: each thread then
    // reads back only the g and 1/S it wrote itself
    const double Lam = pixel_tables<double, BTT>(m, V.g, nullptr, nullptr, red);
    const double c = exp(-Lam);
    row_normalisers<double, BTT>(n, V.g, c, V.u, V.invs, red);
    constexpr bool RT = E <= 8;  // g and 1/S in registers
    constexpr int ER = RT ? E : 1;
    const double* gp = V.g + j0;
    const double* ip = V.invs + j0;
    double gv[ER], iv[ER], xv[E], dv[E], yv[E];
    double sum = 0.0, bad = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool own = e < cnt;
      if constexpr (RT) {
        gv[e] = own ? gp[e] : 0.0;
        iv[e] = own ? ip[e] : 0.0;
      }
      xv[e] = own ? static_cast<double>(xbuf[m.vec_off + j0 + e]) : 0.0;
      if (own) {
        if (!(xv[e] >= 0.0) || !isfinite(xv[e])) bad += 1.0;
        else sum += xv[e];
      }
    }
    block_sum2<BTT>(sum, bad, red);
    // the iterate as power_start takes it: normalised, or uniform if unusable
    const bool usable = bad == 0.0 && sum > 0.0 && isfinite(sum);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      xv[e] = usable ? xv[e] / sum : 1.0 / n;
      dv[e] = 0.0;
      if (e < cnt) xs[tail_slot<E>(j0 + e)] = xv[e];
    }
    __syncthreads();
    // the remaining sweeps of this start (the iterate is not re-run from
    // uniform when they run out, whatever the start was)
    stop_init(st, 0, 0);
    KOpts oc = o;
    oc.max_iter = o.max_iter - prev.iter;
    const int l = m.l;
    const double f = m.frac;
    for (;;) {
      double cs = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (e < cnt) {
          int i = j0 + e - l;
          if (i < 0) i += n;
          double xi = xs[tail_slot<E>(i)];
          if (f != 0.0) xi = (1.0 - f) * xi + f * xs[tail_slot<E>(i == 0 ? n - 1 : i - 1)];
          yv[e] = xi * (RT ? iv[e % ER] : ip[e]);
          cs += yv[e];
        }
      }
      double tot;
      double U = block_exclusive_scan<BTT>(cs, red, tot);  // every read of xs is done after it
      double sy = 0.0, rs = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (e < cnt) {
          U += yv[e];
          yv[e] = (RT ? gv[e % ER] : gp[e]) * (c * tot + (1.0 - c) * U);
          sy += yv[e];
          rs += fabs(yv[e] - xv[e]);
        }
      }
      block_sum2<BTT>(sy, rs, red);
      double chg = 0.0, dd = 0.0, ddp = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (e < cnt) {
          const double xn = yv[e] / sy;
          const double d = xn - xv[e];
          chg += fabs(d);
          dd += d * d;
          ddp += d * dv[e];
          dv[e] = d;
          xv[e] = xn;
          xs[tail_slot<E>(j0 + e)] = xn;
        }
      }
      block_sum3<BTT>(chg, dd, ddp, red);  // its barriers publish the new xs
      const bool restart = stop_update(st, oc, chg, dd, ddp, rs, true, 1.1102230246251565e-16);
      if (restart) {  // the same on every thread: the sums are the block's
#pragma unroll
        for (int e = 0; e < E; ++e) {
          xv[e] = 1.0 / n;
          dv[e] = 0.0;
          if (e < cnt) xs[tail_slot<E>(j0 + e)] = xv[e];
        }
        __syncthreads();
      }
      if (st.done) break;
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (e < cnt) pi_packed[m.pi_off + j0 + e] = static_cast<T>(xv[e]);
    st.total_iter += prev.total_iter;
    st.flags |= prev.flags & (DTM_INFO_WARM_REJECTED | DTM_INFO_RESTARTED);
  }
  st.flags |= DTM_INFO_CONTINUED;
  if (threadIdx.x == 0) {
    dtm_solve_info info = make_info(st);
    info.dense_sweeps = prev.total_iter;
    infos[m.index] = info;
    states[q].s = st;
  }
}

// IN_LDS: the five vectors the iteration touches (g, 1/S, x, u, the last
// difference) live in LDS (5 n doubles, n <= kLdsMaxN) instead of the
// workspace, so every pass over them is an LDS pass.
template <typename T, bool IN_LDS>
__global__ __launch_bounds__(BT) void k_solve_factored(const PixelMeta* __restrict__ metas,
                                                       double* __restrict__ fact, int64_t vec_elems,
                                                       const T* __restrict__ x0_packed,
                                                       T* __restrict__ pi_packed,
                                                       dtm_solve_info* __restrict__ infos, KOpts o) {
  __shared__ double red[3 * BT / kWave];
  extern __shared__ double lds_vec[];
  const PixelMeta m = metas[blockIdx.x];
  Vecs V = vecs(fact, vec_elems, m);
  if constexpr (IN_LDS) {
    V.g = lds_vec;
    V.invs = lds_vec + m.n;
    V.x = lds_vec + 2 * m.n;
    V.u = lds_vec + 3 * m.n;
    V.dp = lds_vec + 4 * m.n;
  }
  const double c = tables(m, V, red);
  const StopState st = power<T>(m, V, c, x0_packed ? x0_packed + m.pi_off : nullptr, o, red);
  int j0, j1;
  chunk_of(m.n, j0, j1);
  for (int j = j0; j < j1; ++j) pi_packed[m.pi_off + j] = static_cast<T>(V.x[j]);
  if (threadIdx.x == 0) {
    dtm_solve_info info = make_info(st);
    info.dense_sweeps = 0;  // no matrix is stored
    infos[m.index] = info;
  }
}

// ============================================================================
// One wavefront per pixel (n <= 64 E): lane t owns bins [t E, t E + E); its
// tables, the last difference and the product stay in registers, and the
// iterate lives in LDS, for the shifted reads of the next product.  The LDS
// copy pads one slot after every E bins, so the lanes' strided accesses fall
// in distinct banks.  Scans and sums are wavefront shuffles, so no block
// barrier is ever needed and the four pixels of a block run independently.
// Same steps and stop rule as k_solve_factored.
// ============================================================================

namespace wave {

// Exclusive prefix over the lanes of v; *total gets the sum of all lanes.
// The exclusive value is the previous lane's inclusive one, not the
// inclusive one minus v: a small prefix next to a large v keeps its digits.
__device__ inline double excl_scan(double v, int lane, double* total) {
  double s = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const double u = __shfl_up(s, d, kWave);
    if (lane >= d) s += u;
  }
  *total = __shfl(s, kWave - 1, kWave);
  const double prev = __shfl_up(s, 1, kWave);
  return lane == 0 ? 0.0 : prev;
}

// Exclusive suffix over the lanes of v (sum over the lanes after this one),
// taken from the next lane's inclusive suffix.
__device__ inline double excl_scan_rev(double v, int lane) {
  double s = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const double u = __shfl_down(s, d, kWave);
    if (lane + d < kWave) s += u;
  }
  const double next = __shfl_down(s, 1, kWave);
  return lane == kWave - 1 ? 0.0 : next;
}

__device__ inline void sync_wave() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// LDS slot of bin i: one pad slot after every E bins.
template <int E>
__device__ inline int slot(int i) {
  return i + i / E;
}

template <int E>
constexpr size_t lds_doubles() {
  return static_cast<size_t>(kWave) * (E + 1);
}

// Where the spectral analysis wants a pixel's float64 tables and pi (the
// vectors g, 1/S and x of its scratch, c per pixel) and its mixing steps
// reset: set for the first stage of dtm_spectral_batched, null otherwise.
struct SpecOut {
  double* fact;
  int64_t vec_elems;
  double* scal;
  dtm_spectral_info* out;
};

template <typename T, int E, bool SPEC = false>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(2))) void k_solve_factored_wave(const PixelMeta* __restrict__ metas, int n_pixels,
                                                            const T* __restrict__ x0_packed,
                                                            T* __restrict__ pi_packed,
                                                            dtm_solve_info* __restrict__ infos, KOpts o,
                                                            SpecOut so) {
  extern __shared__ double lds_x[];
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int p = blockIdx.x * (BT / kWave) + wid;
  if (p >= n_pixels) return;  // whole wavefronts only; nothing below waits for another wavefront
  const PixelMeta m = metas[p];
  const int n = m.n;
  double* xs = lds_x + wid * 2 * lds_doubles<E>();
  const int j0 = lane * E;
  double* xo = xs + slot<E>(j0);  // this lane's own bins (E consecutive slots)

  // ---- bin tables (as pixel_tables and row_normalisers, per wavefront) ----
  // The flux integrals of the bins are taken with bin j = 64 q + lane (q < E)
  // so that the bins near the pulse, the only ones whose normal tails are not
  // exactly zero (erfc(40 / sqrt 2) / 2 underflows, and so does the pulse
  // term of lambda there), are spread over all lanes; a far bin takes those
  // exact zeros without calling erfc or exp.  The integrals then pass through
  // LDS to the lane that owns the bin, which sums them in bin order as
  // pixel_tables does.  The second LDS copy per wavefront serves only this
  // transposition; the kernel is held to two wavefronts per SIMD so that the
  // tables' registers do not halve its residency.
  constexpr double kFar = 40.0;
  const double delta = m.t_r / n, is = 1.0 / m.sigma, bq = m.B / m.t_r;
  double* ts = xs + lds_doubles<E>();  // second LDS copy, used by the tables only
  double dF[E], sh[E], lam[E];  // integral over the bin, S x normal mass up to its centre, lambda at the centre
#pragma unroll 2
  for (int q = 0; q < E; ++q) {
    const int j = q * kWave + lane;
    if (j < n) {
      const double zl = (j * delta - m.tau) * is;
      const double zm = (j * delta + 0.5 * delta - m.tau) * is, zh = ((j + 1) * delta - m.tau) * is;
      double mh = 0.0, mf = 0.0;
      if (zh >= -kFar && zl <= kFar) {
        const double tl = gauss_tail(zl), tm = gauss_tail(zm), th = gauss_tail(zh);
        mh = mass_from_tails(zl, tl, zm, tm);
        mf = mass_from_tails(zl, tl, zh, th);
      }
      xs[slot<E>(j)] = m.S * mf + bq * delta;
      ts[slot<E>(j)] = m.S * mh;
    }
  }
  sync_wave();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    dF[e] = (j0 + e < n) ? xo[e] : 0.0;
    sh[e] = (j0 + e < n) ? ts[slot<E>(j0 + e)] : 0.0;
  }
  sync_wave();
#pragma unroll 2
  for (int q = 0; q < E; ++q) {
    const int j = q * kWave + lane;
    if (j < n) {
      const double zl = (j * delta - m.tau) * is, zh = ((j + 1) * delta - m.tau) * is;
      xs[slot<E>(j)] = (m.lam_mode == 0 && zh >= -kFar && zl <= kFar) ? flux_at(m, j * delta + 0.5 * delta) : bq;
    }
  }
  sync_wave();
#pragma unroll
  for (int e = 0; e < E; ++e) lam[e] = (j0 + e < n) ? xo[e] : 0.0;
  sync_wave();
  const int jb = min(j0, n), je = min(j0 + E, n);
  const double zb = (jb * delta - m.tau) * is, ze = (je * delta - m.tau) * is;
  double part = 0.0;
  if (je > jb) {
    const double mass = (ze >= -kFar && zb <= kFar) ? mass_from_tails(zb, gauss_tail(zb), ze, gauss_tail(ze)) : 0.0;
    part = m.S * mass + bq * ((je - jb) * delta);
  }
  double Lam;
  double acc = excl_scan(part, lane, &Lam);
  double g[E], inv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    g[e] = 0.0;
    if (j0 + e < n) {
      const double F = acc + sh[e] + bq * (0.5 * delta);
      if (m.lam_mode == 0) g[e] = lam[e] * exp(-F);
      else if (m.lam_mode == 1) g[e] = dF[e] / delta * exp(-F);
      else g[e] = exp(-acc) * -expm1(-dF[e]) / delta;
      acc += dF[e];
    }
  }
  const double c = exp(-Lam);
  {
    double cs = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) cs += g[e];
    double tot;
    double P = excl_scan(cs, lane, &tot);
    double Tk = excl_scan_rev(cs, lane);
    // inv[] first holds the exclusive prefixes p_k, then 1 / (T_k + c p_k)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      inv[e] = P;
      P += g[e];
    }
#pragma unroll
    for (int e = E - 1; e >= 0; --e) {
      Tk += g[e];
      inv[e] = (j0 + e < n) ? 1.0 / (Tk + c * inv[e]) : 0.0;
    }
  }

  // ---- start vector ---------------------------------------------------------
  StopState st;
  stop_init(st, 0, 0);
  const T* x0 = x0_packed ? x0_packed + m.pi_off : nullptr;
  double sum = 0.0, bad = 0.0;
  if (x0) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (j0 + e < n) {
        const double v = static_cast<double>(x0[j0 + e]);
        if (!(v >= 0.0) || !isfinite(v)) bad += 1.0;
        else sum += v;
      }
    sum = wave_sum(sum);
    bad = wave_sum(bad);
  }
  const bool warm = x0 && bad == 0.0 && sum > 0.0 && isfinite(sum);
  if (x0 && !warm) st.flags |= DTM_INFO_WARM_REJECTED;
  st.warm = warm ? 1 : 0;
  double dp[E], y[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = j0 + e;
    if (j < n) xo[e] = warm ? static_cast<double>(x0[j]) / sum : 1.0 / n;
    dp[e] = 0.0;
  }
  sync_wave();

  // ---- power iteration --------------------------------------------------------
  // bin k reads x_{k - l} (and x_{k - l - 1} for an interpolated shift); the
  // lane's first read index, the rest follow with one wrap at most
  int i0 = j0 - m.l;
  if (i0 < 0) i0 += n;
  const double f = m.frac;
  for (;;) {
    // u_k = x_{k - l} / S_k into y[]
    double cs = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      y[e] = 0.0;
      if (j0 + e < n) {
        int i = i0 + e;
        if (i >= n) i -= n;
        double xv = xs[slot<E>(i)];
        if (f != 0.0) {
          const int i2 = i == 0 ? n - 1 : i - 1;
          xv = (1.0 - f) * xv + f * xs[slot<E>(i2)];
        }
        y[e] = xv * inv[e];
        cs += y[e];
      }
    }
    double tot;
    double U = excl_scan(cs, lane, &tot);
    // y_j = g_j (c U_{n-1} + (1 - c) U_j), in place of u
    double sy = 0.0, rs = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (j0 + e < n) {
        U += y[e];
        y[e] = g[e] * (c * tot + (1.0 - c) * U);
        sy += y[e];
        rs += fabs(y[e] - xo[e]);
      }
    }
    sy = wave_sum(sy);
    rs = wave_sum(rs);
    sync_wave();  // every shifted read of xs is done before the writes below
    const double isy = 1.0 / sy;
    double ch = 0.0, dd = 0.0, ddp = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (j0 + e < n) {
        const double xn = y[e] * isy;
        const double d = xn - xo[e];
        ch += fabs(d);
        dd += d * d;
        ddp += d * dp[e];
        dp[e] = d;
        xo[e] = xn;
      }
    }
    ch = wave_sum(ch);
    dd = wave_sum(dd);
    ddp = wave_sum(ddp);
    const bool restart = stop_update(st, o, ch, dd, ddp, rs, true, 1.1102230246251565e-16);
    if (restart) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (j0 + e < n) xo[e] = 1.0 / n;
        dp[e] = 0.0;
      }
    }
    sync_wave();  // the new iterate is in xs before the next shifted reads
    if (st.done) break;
  }
  if constexpr (SPEC) {
    // the spectral analysis' first stage: tables and pi into its scratch
    double* base = so.fact + m.vec_off;
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (j0 + e < n) {
        base[j0 + e] = g[e];
        base[so.vec_elems + j0 + e] = inv[e];
        base[2 * so.vec_elems + j0 + e] = xo[e];
      }
    if (lane == 0) {
      so.scal[p] = c;
      so.out[m.index].mixing_steps = -1;
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (j0 + e < n) pi_packed[m.pi_off + j0 + e] = static_cast<T>(xo[e]);
    if (lane == 0) {
      dtm_solve_info info = make_info(st);
      info.dense_sweeps = 0;  // no matrix is stored
      infos[m.index] = info;
    }
  }
}

}  // namespace wave

// Deflated operator A v = v P~ - (v . 1) pi (removes the Perron pair: left
// eigenvectors of the other eigenvalues are orthogonal to the right Perron
// vector 1), given s = v . 1.  out may alias V.u.
__device__ void deflated(const PixelMeta& m, const Vecs& V, double c, const double* v, double s, double* out,
                         double* red) {
  int j0, j1;
  chunk_of(m.n, j0, j1);
  apply(m.n, m.l, m.frac, v, V.g, V.invs, c, V.u, out, red);
  if (s != 0.0)
    for (int j = j0; j < j1; ++j) out[j] -= s * V.x[j];
  __syncthreads();
}

// Exclusive prefix sums over the block, in thread order, of N values at
// once (one barrier round for all); tot gets the N totals.  red holds
// N * BT / 64 doubles.
template <int N>
__device__ inline void block_exclusive_scan_n(double (&v)[N], double (&tot)[N], double* red) {
  constexpr int NW = BT / kWave;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  double x[N], excl[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    x[q] = v[q];
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const double y = __shfl_up(x[q], off, kWave);
      if (lane >= off) x[q] += y;
    }
    excl[q] = __shfl_up(x[q], 1, kWave);
    if (lane == 0) excl[q] = 0.0;
  }
  __syncthreads();
  if (lane == kWave - 1) {
#pragma unroll
    for (int q = 0; q < N; ++q) red[q * NW + w] = x[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double base = 0.0, t = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      if (i < w) base += red[q * NW + i];
      t += red[q * NW + i];
    }
    v[q] = base + excl[q];
    tot[q] = t;
  }
}

// The deflated operator on the first cnt of N vectors at once: Y[i] =
// X[i] P~ - s[i] pi, each product by the factored form of apply(), all N
// prefix scans in one block scan.  Y[i] must not alias any X.  Ends with a
// block barrier.
template <int N>
__device__ void deflated_n(const PixelMeta& m, const Vecs& V, double c, double* const (&X)[N],
                           const double (&s)[N], double* const (&Y)[N], int cnt, double* red) {
  const int n = m.n;
  int j0, j1;
  chunk_of(n, j0, j1);
  double cs[N];
#pragma unroll
  for (int q = 0; q < N; ++q) cs[q] = 0.0;
  for (int k = j0; k < j1; ++k) {
    int i = k - m.l;
    if (i < 0) i += n;
    const int i2 = i == 0 ? n - 1 : i - 1;
    const double ik = V.invs[k];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      if (q < cnt) {
        const double xk = m.frac == 0.0 ? X[q][i] : (1.0 - m.frac) * X[q][i] + m.frac * X[q][i2];
        const double u = xk * ik;
        Y[q][k] = u;
        cs[q] += u;
      }
    }
  }
  double tot[N];
  block_exclusive_scan_n<N>(cs, tot, red);
#pragma unroll
  for (int q = 0; q < N; ++q) {
    if (q < cnt) {
      double U = cs[q];
      for (int j = j0; j < j1; ++j) {
        U += Y[q][j];
        Y[q][j] = V.g[j] * (c * tot[q] + (1.0 - c) * U) - s[q] * V.x[j];
      }
    }
  }
  __syncthreads();
}

// Sums of N values over the block (every thread gets all of them), one
// barrier round for all; red holds N * BT / 64 doubles.
template <int N>
__device__ inline void block_sum_n(double (&v)[N], double* red) {
  constexpr int NW = BT / kWave;
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = wave_sum(v[q]);
  __syncthreads();
  if ((threadIdx.x % kWave) == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) red[q * NW + w] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) t += red[q * NW + i];
    v[q] = t;
  }
}

// ---- eigenvalues of a small dense matrix (the Rayleigh-Ritz step) --------
// Real k x k matrix h (row-major, k <= KSUB, overwritten) -> its k
// eigenvalues (er, ei).  Householder reduction to upper Hessenberg form,
// then the shifted QR algorithm in complex arithmetic on the unreduced
// trailing block: each step factors A - mu I = QR by Givens rotations and
// forms RQ + mu I, with mu the eigenvalue of the trailing 2 x 2 block nearer
// its last diagonal entry (an exceptional shift every eleventh step without
// a deflation); a subdiagonal entry below unit round-off relative to its
// diagonal neighbours splits the block.  ar, ai: k x k scratch.  Returns
// false when a block did not split within 60 steps (the diagonal is then
// taken as it stands).  Run by one thread.
struct Cx {
  double re, im;
};
__device__ inline Cx cx_mul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Cx cx_sqrt(Cx z) {
  const double r = hypot(z.re, z.im);
  if (r == 0.0) return {0.0, 0.0};
  const double t = sqrt(0.5 * (r + fabs(z.re)));
  if (z.re >= 0.0) return {t, z.im / (2.0 * t)};
  return {fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}
__device__ inline double cx_abs(Cx z) { return hypot(z.re, z.im); }

__device__ bool small_eigvals(double* h, int k, double* ar, double* ai, double* er, double* ei) {
  for (int j = 0; j + 2 < k; ++j) {
    double v[KSUB];
    double alpha = 0.0;
    for (int i = j + 1; i < k; ++i) alpha += h[i * k + j] * h[i * k + j];
    alpha = sqrt(alpha);
    if (alpha == 0.0) continue;
    if (h[(j + 1) * k + j] > 0.0) alpha = -alpha;
    double vn = 0.0;
    for (int i = j + 1; i < k; ++i) {
      v[i - j - 1] = h[i * k + j] - (i == j + 1 ? alpha : 0.0);
      vn += v[i - j - 1] * v[i - j - 1];
    }
    if (vn == 0.0) continue;
    const double f = 2.0 / vn;
    for (int col = 0; col < k; ++col) {  // rows j+1.. from the left
      double t = 0.0;
      for (int i = j + 1; i < k; ++i) t += v[i - j - 1] * h[i * k + col];
      t *= f;
      for (int i = j + 1; i < k; ++i) h[i * k + col] -= t * v[i - j - 1];
    }
    for (int row = 0; row < k; ++row) {  // columns j+1.. from the right
      double t = 0.0;
      for (int i = j + 1; i < k; ++i) t += h[row * k + i] * v[i - j - 1];
      t *= f;
      for (int i = j + 1; i < k; ++i) h[row * k + i] -= t * v[i - j - 1];
    }
  }
  for (int i = 0; i < k * k; ++i) {
    ar[i] = h[i];
    ai[i] = 0.0;
  }
  const auto at = [&](int r, int c) { return Cx{ar[r * k + c], ai[r * k + c]}; };
  const auto put = [&](int r, int c, Cx z) {
    ar[r * k + c] = z.re;
    ai[r * k + c] = z.im;
  };
  constexpr double eps = 1.1102230246251565e-16;
  bool ok = true;
  int hi = k - 1, steps = 0;
  while (hi >= 0) {
    if (hi == 0) {
      er[0] = ar[0];
      ei[0] = ai[0];
      break;
    }
    int lo = hi;
    while (lo > 0 && cx_abs(at(lo, lo - 1)) > eps * (cx_abs(at(lo - 1, lo - 1)) + cx_abs(at(lo, lo)))) --lo;
    if (lo == hi || steps >= 60) {
      if (lo != hi) ok = false;
      er[hi] = ar[hi * k + hi];
      ei[hi] = ai[hi * k + hi];
      --hi;
      steps = 0;
      continue;
    }
    const Cx a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
    Cx mu;
    if (steps > 0 && steps % 11 == 0) {
      mu = {d.re + cx_abs(c), d.im};
    } else {
      const Cx half = {0.5 * (a.re - d.re), 0.5 * (a.im - d.im)};
      const Cx hh = cx_mul(half, half), bc = cx_mul(b, c);
      const Cx disc = cx_sqrt({hh.re + bc.re, hh.im + bc.im});
      const Cx m1 = {d.re + half.re + disc.re, d.im + half.im + disc.im};
      const Cx m2 = {d.re + half.re - disc.re, d.im + half.im - disc.im};
      mu = cx_abs({m1.re - d.re, m1.im - d.im}) <= cx_abs({m2.re - d.re, m2.im - d.im}) ? m1 : m2;
    }
    ++steps;
    for (int i = lo; i <= hi; ++i) put(i, i, {ar[i * k + i] - mu.re, ai[i * k + i] - mu.im});
    Cx cs[KSUB], sn[KSUB];
    for (int i = lo; i < hi; ++i) {  // R = G_{hi-1} ... G_lo (A - mu I)
      const Cx x = at(i, i), y = at(i + 1, i);
      const double r = hypot(cx_abs(x), cx_abs(y));
      const Cx cc = r == 0.0 ? Cx{1.0, 0.0} : Cx{x.re / r, x.im / r};
      const Cx ss = r == 0.0 ? Cx{0.0, 0.0} : Cx{y.re / r, y.im / r};
      cs[i] = cc;
      sn[i] = ss;
      const Cx ccc = {cc.re, -cc.im}, ssc = {ss.re, -ss.im};
      for (int col = i; col <= hi; ++col) {
        const Cx u = at(i, col), w = at(i + 1, col);
        const Cx p = cx_mul(ccc, u), q = cx_mul(ssc, w), s1 = cx_mul(ss, u), s2 = cx_mul(cc, w);
        put(i, col, {p.re + q.re, p.im + q.im});
        put(i + 1, col, {s2.re - s1.re, s2.im - s1.im});
      }
    }
    for (int i = lo; i < hi; ++i) {  // R G_lo^H ... G_{hi-1}^H
      const Cx cc = cs[i], ss = sn[i];
      const Cx ccc = {cc.re, -cc.im}, ssc = {ss.re, -ss.im};
      const int rmax = min(i + 2, hi);
      for (int row = lo; row <= rmax; ++row) {
        const Cx u = at(row, i), w = at(row, i + 1);
        const Cx p = cx_mul(u, cc), q = cx_mul(w, ss), s1 = cx_mul(u, ssc), s2 = cx_mul(w, ccc);
        put(row, i, {p.re + q.re, p.im + q.im});
        put(row, i + 1, {s2.re - s1.re, s2.im - s1.im});
      }
    }
    for (int i = lo; i <= hi; ++i) put(i, i, {ar[i * k + i] + mu.re, ai[i * k + i] + mu.im});
  }
  return ok;
}

// Start vector number i of the subspace: a fixed non-symmetric pattern.
__device__ inline double start_pattern(int i, int j) {
  return 1.0 + 0.5 * sin((0.7 + 0.37 * i) * j + 0.3 * i) + ((j * 7919 + i * 104729) % 13) * 0.01;
}

// First stage of the spectral analysis, one block per pixel: the float64
// tables and pi (power iteration on the factored product) into the scratch,
// c = e^{-Lambda} into scal_out, and the pixel's mixing steps set to -1 (the
// mixing search merges its result into them).  The subspace search and the
// mixing search both start from these and run side by side.
__global__ __launch_bounds__(BT) void k_spectral_pi(const PixelMeta* __restrict__ metas,
                                                    double* __restrict__ fact, int64_t vec_elems,
                                                    double* __restrict__ scal_out,
                                                    dtm_spectral_info* __restrict__ out, KOpts o) {
  __shared__ double red[3 * BT / kWave];
  const PixelMeta m = metas[blockIdx.x];
  const Vecs V = vecs(fact, vec_elems, m);
  const double c = tables(m, V, red);
  power<double>(m, V, c, static_cast<const double*>(nullptr), o, red);  // pi -> V.x
  if (threadIdx.x == 0) {
    scal_out[blockIdx.x] = c;
    out[m.index].mixing_steps = -1;
  }
}

// lambda_2 of the dead-time matrix (Section 4): orthogonal iteration on the
// deflated operator A v = v P~ - (v . 1) pi with a KSUB-dimensional subspace
// (min(KSUB, n - 1) vectors), each step
//   Q = orthonormal basis of W (classical Gram-Schmidt, two passes),
//   W = A Q,  H = Q^T W  (the Rayleigh quotient of the subspace),
// whose eigenvalues (Ritz values) approach the KSUB eigenvalues of largest
// modulus of A, i.e. lambda_2, lambda_3, ... of P~: the one of largest
// modulus converges at the rate |lambda_{KSUB+2} / lambda_2| per step, so
// eigenvalues close to lambda_2 in modulus (a near-tie with lambda_3) do not
// slow it.  The Rayleigh-Ritz step is taken every eighth step until two of
// them agree to 1e-9, then every step; the search stops when lambda_2 has
// changed by at most 1e-13 (1 + |lambda_2|) and the next modulus by at most
// 1e-11 (1 + |lambda_2|) in two successive steps, or after max_iter steps.  A basis vector that A
// annihilates (its orthogonalised norm below 1e-14 of its norm) stays zero.
// Starts from the tables, pi and c of the first stage (k_spectral_pi, or the
// wavefront solver up to 1024 bins); writes every field of the pixel's
// report but mixing_steps.  IN_LDS: g, 1/S, pi and the 2 KSUB subspace
// vectors live in LDS (n <= kSpecLdsMaxN).
template <bool IN_LDS>
__global__ __launch_bounds__(BT) void k_spectral(const PixelMeta* __restrict__ metas,
                                                 double* __restrict__ fact, int64_t vec_elems,
                                                 const double* __restrict__ scal,
                                                 dtm_spectral_info* __restrict__ out, int max_iter) {
  __shared__ double red[KSUB * KSUB * BT / kWave];
  __shared__ double hs[KSUB * KSUB], har[KSUB * KSUB], hai[KSUB * KSUB], er[KSUB], ei[KSUB];
  __shared__ int eig_ok;
  extern __shared__ double lds_vec[];
  const PixelMeta m = metas[blockIdx.x];
  const int n = m.n;
  const Vecs G = vecs(fact, vec_elems, m);
  Vecs V = G;
  double* Q[KSUB];
  double* W[KSUB];
  {
    double* base = IN_LDS ? lds_vec : fact + m.vec_off;
    const int64_t stride = IN_LDS ? static_cast<int64_t>(n) : vec_elems;
    // the search uses g, 1/S and pi of the solver's five vectors
    const int first = IN_LDS ? 3 : 5;
    if constexpr (IN_LDS) {
      V.g = base;
      V.invs = base + stride;
      V.x = base + 2 * stride;
      V.u = V.dp = nullptr;
    }
#pragma unroll
    for (int i = 0; i < KSUB; ++i) {
      Q[i] = base + (first + i) * stride;
      W[i] = base + (first + KSUB + i) * stride;
    }
  }
  const double c = scal[blockIdx.x];
  int j0, j1;
  chunk_of(n, j0, j1);
  if constexpr (IN_LDS) {
    for (int j = j0; j < j1; ++j) {
      V.g[j] = G.g[j];
      V.invs[j] = G.invs[j];
      V.x[j] = G.x[j];
    }
    __syncthreads();
  }
  const int ke = min(KSUB, n - 1);
  {
    double sums[KSUB];
#pragma unroll
    for (int i = 0; i < KSUB; ++i) {
      sums[i] = 0.0;
      if (i < ke)
        for (int j = j0; j < j1; ++j) {
          const double v = start_pattern(i, j);
          Q[i][j] = v;
          sums[i] += v;
        }
    }
    block_sum_n<KSUB>(sums, red);
    deflated_n<KSUB>(m, V, c, Q, sums, W, ke, red);
  }
  double re = 0.0, im = 0.0, l3 = 0.0, change = 0.0, prev_re = 2.0, prev_im = 2.0, prev_l3 = 2.0;
  int it = 0, settled = 0, flags = 0;
  bool all_ok = true;
  int next_rr = 8;     // step count at which the next Rayleigh-Ritz step is taken
  bool fine = false;   // Ritz values within 1e-9 of settling: take one every step
  for (; it < max_iter; ++it) {
    // Q = orthonormal basis of W: two classical Gram-Schmidt passes; the
    // second pass's reduction also gives ||v||^2 and sum(v), from which the
    // norm and sum after its projection follow (the q_a are orthonormal:
    // ||v - sum d_a q_a||^2 = ||v||^2 - sum d_a^2)
    double s[KSUB];
#pragma unroll
    for (int i = 0; i < KSUB; ++i) {
      s[i] = 0.0;
      if (i >= ke) continue;
      for (int j = j0; j < j1; ++j) Q[i][j] = W[i][j];
      double n0 = 0.0, nrm2 = 0.0, sum = 0.0;
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        double d[KSUB + 2];
#pragma unroll
        for (int a = 0; a < KSUB + 2; ++a) d[a] = 0.0;
        for (int j = j0; j < j1; ++j) {
          const double qi = Q[i][j];
#pragma unroll
          for (int a = 0; a < KSUB; ++a)
            if (a < i) d[a] += Q[a][j] * qi;
          d[KSUB] += qi * qi;
          d[KSUB + 1] += qi;
        }
        block_sum_n<KSUB + 2>(d, red);
        if (pass == 0) {
          n0 = d[KSUB];
        } else {
          nrm2 = d[KSUB];
          sum = d[KSUB + 1];
#pragma unroll
          for (int a = 0; a < KSUB; ++a)
            if (a < i) {
              nrm2 -= d[a] * d[a];
              sum -= d[a] * s[a];
            }
        }
        for (int j = j0; j < j1; ++j) {
          double v = Q[i][j];
#pragma unroll
          for (int a = 0; a < KSUB; ++a)
            if (a < i) v -= d[a] * Q[a][j];
          Q[i][j] = v;
        }
      }
      const double sc = (nrm2 > 1e-28 * n0 && nrm2 > 0.0) ? 1.0 / sqrt(nrm2) : 0.0;
      for (int j = j0; j < j1; ++j) Q[i][j] *= sc;
      s[i] = sum * sc;
      __syncthreads();
    }
    // W = A Q
    deflated_n<KSUB>(m, V, c, Q, s, W, ke, red);
    // Rayleigh-Ritz every eighth step until the Ritz values have nearly
    // settled, then every step
    if (!fine && it + 1 < next_rr && it + 1 < max_iter) continue;
    double h[KSUB * KSUB];
#pragma unroll
    for (int e = 0; e < KSUB * KSUB; ++e) h[e] = 0.0;
    for (int j = j0; j < j1; ++j) {
#pragma unroll
      for (int a = 0; a < KSUB; ++a)
#pragma unroll
        for (int b = 0; b < KSUB; ++b)
          if (a < ke && b < ke) h[a * KSUB + b] += Q[a][j] * W[b][j];
    }
    block_sum_n<KSUB * KSUB>(h, red);
    if (threadIdx.x == 0) {
      for (int a = 0; a < ke; ++a)
        for (int b = 0; b < ke; ++b) hs[a * ke + b] = h[a * KSUB + b];
      eig_ok = small_eigvals(hs, ke, har, hai, er, ei) ? 1 : 0;
    }
    __syncthreads();
    if (!eig_ok) all_ok = false;
    // lambda_2: the Ritz value of largest modulus; lambda_3: the largest of
    // the others, leaving out lambda_2's conjugate
    int i2 = 0;
    for (int i = 1; i < ke; ++i)
      if (hypot(er[i], ei[i]) > hypot(er[i2], ei[i2])) i2 = i;
    re = er[i2];
    im = fabs(ei[i2]);
    const double a2 = hypot(re, im);
    if (im <= 1e-13 * (1.0 + a2)) im = 0.0;  // a real eigenvalue, up to the rounding of the QR steps
    int partner = -1;
    if (im > 0.0)
      for (int i = 0; i < ke; ++i)
        if (i != i2 && partner < 0 && hypot(er[i] - er[i2], ei[i] + ei[i2]) <= 1e-9 * (1.0 + a2)) partner = i;
    l3 = 0.0;
    for (int i = 0; i < ke; ++i)
      if (i != i2 && i != partner) l3 = fmax(l3, hypot(er[i], ei[i]));
    const double ch2 = hypot(re - prev_re, im - prev_im), ch3 = fabs(l3 - prev_l3);
    change = fmax(ch2, ch3);
    prev_re = re;
    prev_im = im;
    prev_l3 = l3;
    __syncthreads();  // every thread has read er / ei before the next step writes them
    if (!fine) {
      fine = change <= 1e-9 * (1.0 + a2);
      next_rr = it + 1 + 8;
      continue;
    }
    settled = (ch2 <= 1e-13 * (1.0 + a2) && ch3 <= 1e-11 * (1.0 + a2)) ? settled + 1 : 0;
    if (settled >= 2) break;
  }
  if (settled < 2) flags |= DTM_SPECTRAL_UNSETTLED;
  if (!all_ok) flags |= DTM_SPECTRAL_UNSETTLED;
  if (l3 >= (1.0 - 1e-9) * hypot(re, im) && l3 > 0.0) flags |= DTM_SPECTRAL_TIED;
  if (threadIdx.x == 0) {
    // field by field: the mixing search may be merging into mixing_steps
    dtm_spectral_info& si = out[m.index];
    si.lambda2_re = re;
    si.lambda2_im = im;
    si.lambda2_abs = hypot(re, im);
    si.lambda2_arg = atan2(im, re);
    si.lambda3_abs = l3;
    si.ritz_change = change;
    si.iterations = min(it + 1, max_iter);
    si.flags = flags;
    si.reserved = 0;
  }
}

// Empirical mixing steps: every start state e_s advanced on its own, one
// thread per start state (each thread runs its own prefix scan over the n
// bins); flat pixel-major grid, block y of a pixel owns states
// [y BT, (y + 1) BT).  X and Y are
// n x n, stored state-minor (X[k * n + s]) so that a wavefront reads
// consecutive states.  The distance of each start state from pi does not
// grow from one step to the next (P~ is stochastic), so the pixel mixes at
// the largest over its states of the first step within eps: each block stops
// when all its states are within eps and merges its step by atomicMax (a
// block that runs out of steps posts max_steps + 1, read as "not reached").
// Requires the tables and pi in V and mixing_steps = -1 (from k_spectral_pi).
__global__ __launch_bounds__(BT) void k_mixing(const PixelMeta* __restrict__ metas,
                                               double* __restrict__ fact, int64_t vec_elems,
                                               double* __restrict__ mix, const int64_t* __restrict__ mix_off,
                                               const double* __restrict__ scal,
                                               dtm_spectral_info* __restrict__ out, double eps,
                                               int max_steps, int state_blocks) {
  __shared__ double red[BT / kWave];
  const int pix = static_cast<int>(blockIdx.x / state_blocks);
  const PixelMeta m = metas[pix];
  const int n = m.n;
  const int s0 = static_cast<int>(blockIdx.x % state_blocks) * BT;
  if (s0 >= n) return;
  const Vecs V = vecs(fact, vec_elems, m);
  const double c = scal[pix];
  double* X = mix + mix_off[pix];
  double* Y = X + static_cast<int64_t>(n) * n;
  const int s = s0 + static_cast<int>(threadIdx.x);
  const bool mine = s < n;
  if (mine)
    for (int k = 0; k < n; ++k) X[static_cast<int64_t>(k) * n + s] = (k == s) ? 1.0 : 0.0;
  int steps = max_steps + 1;
  for (int t = 1; t <= max_steps; ++t) {
    double tv = 0.0;
    if (mine) {
      const auto xs = [X, n, s](int i) { return X[static_cast<int64_t>(i) * n + s]; };
      double tot = 0.0;
#pragma unroll 8
      for (int k = 0; k < n; ++k) tot += shifted_x(xs, n, m.l, m.frac, k) * V.invs[k];
      double U = 0.0;
#pragma unroll 8
      for (int j = 0; j < n; ++j) {
        U += shifted_x(xs, n, m.l, m.frac, j) * V.invs[j];
        const double y = V.g[j] * (c * tot + (1.0 - c) * U);
        Y[static_cast<int64_t>(j) * n + s] = y;
        tv += fabs(y - V.x[j]);
      }
      tv *= 0.5;
    }
    // block max
    for (int off = 32; off > 0; off >>= 1) tv = fmax(tv, __shfl_xor(tv, off, kWave));
    if ((threadIdx.x % kWave) == 0) red[threadIdx.x / kWave] = tv;
    __syncthreads();
    double wmax = 0.0;
    for (int i = 0; i < BT / kWave; ++i) wmax = fmax(wmax, red[i]);
    __syncthreads();
    double* tmp = X;
    X = Y;
    Y = tmp;
    if (wmax <= eps) {
      steps = t;
      break;
    }
  }
  if (threadIdx.x == 0) atomicMax(&out[m.index].mixing_steps, steps);
}

// The same empirical mixing steps with one wavefront per start state (n <= 64
// E): the state's distribution stays on chip, its bins [t E, t E + E) in
// lane t's registers and in a padded LDS copy for the shifted reads, with
// g, 1/S and pi of the pixel in registers; each wavefront stops at its own
// first step within eps and merges it by atomicMax.  Flat pixel-major grid
// (so that each pixel's blocks are dealt to all XCDs): block y of a pixel
// owns states [4 y, 4 y + 4).  No n x n scratch is touched.
template <int E>
__global__ __launch_bounds__(BT) void k_mixing_wave(const PixelMeta* __restrict__ metas,
                                                    const double* __restrict__ fact, int64_t vec_elems,
                                                    const double* __restrict__ scal,
                                                    dtm_spectral_info* __restrict__ out, double eps,
                                                    int max_steps, int state_blocks) {
  extern __shared__ double lds_x[];
  const int pix = static_cast<int>(blockIdx.x / state_blocks);
  const PixelMeta m = metas[pix];
  const int n = m.n;
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int s = static_cast<int>(blockIdx.x % state_blocks) * (BT / kWave) + wid;
  if (s >= n) return;  // whole wavefronts only; nothing below waits for another wavefront
  const double* base = fact + m.vec_off;
  const double* gv = base;
  const double* iv = base + vec_elems;
  const double* pv = base + 2 * vec_elems;
  const double c = scal[pix];
  double* xs = lds_x + wid * wave::lds_doubles<E>();
  const int j0 = lane * E;
  double* xo = xs + wave::slot<E>(j0);
  double g[E], inv[E], pi[E], y[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = j0 + e;
    const bool in = j < n;
    g[e] = in ? gv[j] : 0.0;
    inv[e] = in ? iv[j] : 0.0;
    pi[e] = in ? pv[j] : 0.0;
    if (in) xo[e] = (j == s) ? 1.0 : 0.0;
  }
  wave::sync_wave();
  int i0 = j0 - m.l;
  if (i0 < 0) i0 += n;
  const double f = m.frac;
  int steps = max_steps + 1;
  for (int t = 1; t <= max_steps; ++t) {
    double cs = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      y[e] = 0.0;
      if (j0 + e < n) {
        int i = i0 + e;
        if (i >= n) i -= n;
        double xv = xs[wave::slot<E>(i)];
        if (f != 0.0) {
          const int i2 = i == 0 ? n - 1 : i - 1;
          xv = (1.0 - f) * xv + f * xs[wave::slot<E>(i2)];
        }
        y[e] = xv * inv[e];
        cs += y[e];
      }
    }
    double tot;
    double U = wave::excl_scan(cs, lane, &tot);
    double tv = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (j0 + e < n) {
        U += y[e];
        y[e] = g[e] * (c * tot + (1.0 - c) * U);
        tv += fabs(y[e] - pi[e]);
      }
    }
    tv = 0.5 * wave_sum(tv);
    wave::sync_wave();  // every shifted read of xs is done before the writes below
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (j0 + e < n) xo[e] = y[e];
    wave::sync_wave();
    if (tv <= eps) {
      steps = t;
      break;
    }
  }
  if (lane == 0) atomicMax(&out[m.index].mixing_steps, steps);
}

// Pixels some of whose start states did not mix within max_steps: -1.
__global__ __launch_bounds__(BT) void k_mixing_final(const PixelMeta* __restrict__ metas, int n_pixels,
                                                     dtm_spectral_info* __restrict__ out, int max_steps) {
  const int p = blockIdx.x * BT + threadIdx.x;
  if (p >= n_pixels) return;
  const int idx = metas[p].index;
  if (out[idx].mixing_steps > max_steps) out[idx].mixing_steps = -1;
}

}  // namespace fact
}  // namespace dtm

using namespace dtm;

namespace dtm {

template <typename T, int E>
int launch_tail_reg_e(const dtm_plan* plan, int count, const PixelMeta* metas, const int32_t* sel, double* fact,
                      SolveState* states, void* pi, dtm_solve_info* infos, hipStream_t st) {
  auto kern = fact::k_dense_tail_reg<T, E>;
  constexpr size_t lds = fact::tail_lds_bytes<E>();
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                          static_cast<int>(lds)) != hipSuccess)
    return DTM_EHIP;
  const T* xbuf = reinterpret_cast<const T*>(static_cast<char*>(plan->ws) + plan->off_xbuf);
  hipLaunchKernelGGL(kern, dim3(count), dim3(fact::BTT), lds, st, metas, sel, fact, plan->vec_elems, xbuf, states,
                     static_cast<T*>(pi), infos, plan->kopts);
  return hipGetLastError() == hipSuccess ? DTM_OK : DTM_EHIP;
}

// The continuation of pixels of at most 8192 bins, in 512-thread blocks
// holding ceil(n / 512) <= e bins per thread in registers.
template <typename T>
int launch_tail_reg(const dtm_plan* plan, int e, int count, const PixelMeta* metas, const int32_t* sel,
                    double* fact, SolveState* states, void* pi, dtm_solve_info* infos, hipStream_t st) {
  switch (e) {
    case 2: return launch_tail_reg_e<T, 2>(plan, count, metas, sel, fact, states, pi, infos, st);
    case 4: return launch_tail_reg_e<T, 4>(plan, count, metas, sel, fact, states, pi, infos, st);
    case 8: return launch_tail_reg_e<T, 8>(plan, count, metas, sel, fact, states, pi, infos, st);
    default: return launch_tail_reg_e<T, 16>(plan, count, metas, sel, fact, states, pi, infos, st);
  }
}

int launch_dense_tail(const dtm_plan* plan, int banded, void* pi, dtm_solve_info* infos, void* stream) {
  const int count = static_cast<int>(banded ? plan->big_sel.size() : plan->small_sel.size());
  if (count == 0) return DTM_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(plan->ws);
  const PixelMeta* metas = reinterpret_cast<const PixelMeta*>(w + plan->off_meta);
  const int32_t* sel = reinterpret_cast<const int32_t*>(w + (banded ? plan->off_big : plan->off_small));
  double* fact = reinterpret_cast<double*>(w + plan->off_fact);
  SolveState* states = reinterpret_cast<SolveState*>(w + plan->off_state);
  const int max_n = banded ? plan->max_n_big : plan->max_n_small;
  if (max_n <= fact::BTT * 16) {
    const int e = max_n <= 2 * fact::BTT ? 2 : max_n <= 4 * fact::BTT ? 4 : max_n <= 8 * fact::BTT ? 8 : 16;
    return plan->dt == DTM_F32 ? launch_tail_reg<float>(plan, e, count, metas, sel, fact, states, pi, infos, st)
                               : launch_tail_reg<double>(plan, e, count, metas, sel, fact, states, pi, infos, st);
  }
  if (plan->dt == DTM_F32)
    hipLaunchKernelGGL((fact::k_dense_tail<float>), dim3(count), dim3(fact::BT), 0, st, metas, sel, fact,
                       plan->vec_elems, reinterpret_cast<const float*>(w + plan->off_xbuf), states,
                       static_cast<float*>(pi), infos, plan->kopts);
  else
    hipLaunchKernelGGL((fact::k_dense_tail<double>), dim3(count), dim3(fact::BT), 0, st, metas, sel, fact,
                       plan->vec_elems, reinterpret_cast<const double*>(w + plan->off_xbuf), states,
                       static_cast<double*>(pi), infos, plan->kopts);
  return hipGetLastError() == hipSuccess ? DTM_OK : DTM_EHIP;
}

}  // namespace dtm

extern "C" {

int dtm_solve_factored_batched(const dtm_plan* plan, const void* x0_packed_dev, void* pi_packed_dev,
                               dtm_solve_info* infos_dev, dtm_stream_t stream) {
  if (!plan || !plan->ws || !pi_packed_dev || !infos_dev) return DTM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(plan->ws);
  const PixelMeta* metas = reinterpret_cast<const PixelMeta*>(w + plan->off_meta);
  double* fact = reinterpret_cast<double*>(w + plan->off_fact);
  KOpts o = plan->kopts;
  o.pad = 0;
  if (plan->max_n <= 1024) {
    // one wavefront per pixel, four per block; E bins per lane; two LDS
    // copies of a pixel's bins per wavefront (the iterate, and the tables'
    // second transposition buffer)
    const int E = plan->max_n <= 256 ? 4 : plan->max_n <= 512 ? 8 : 16;
    const dim3 grid((plan->n_pixels + 3) / 4), block(fact::BT);
    const size_t lds = sizeof(double) * 4 * 2 * kWave * (E + 1);
    const void* kern = nullptr;
    if (plan->dt == DTM_F32)
      kern = E == 4 ? reinterpret_cast<const void*>(fact::wave::k_solve_factored_wave<float, 4>)
             : E == 8 ? reinterpret_cast<const void*>(fact::wave::k_solve_factored_wave<float, 8>)
                      : reinterpret_cast<const void*>(fact::wave::k_solve_factored_wave<float, 16>);
    else
      kern = E == 4 ? reinterpret_cast<const void*>(fact::wave::k_solve_factored_wave<double, 4>)
             : E == 8 ? reinterpret_cast<const void*>(fact::wave::k_solve_factored_wave<double, 8>)
                      : reinterpret_cast<const void*>(fact::wave::k_solve_factored_wave<double, 16>);
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
      return DTM_EHIP;
    if (plan->dt == DTM_F32) {
      const float* x0 = static_cast<const float*>(x0_packed_dev);
      float* pi = static_cast<float*>(pi_packed_dev);
      if (E == 4) hipLaunchKernelGGL((fact::wave::k_solve_factored_wave<float, 4>), grid, block, lds, st, metas, plan->n_pixels, x0, pi, infos_dev, o, fact::wave::SpecOut{});
      else if (E == 8) hipLaunchKernelGGL((fact::wave::k_solve_factored_wave<float, 8>), grid, block, lds, st, metas, plan->n_pixels, x0, pi, infos_dev, o, fact::wave::SpecOut{});
      else hipLaunchKernelGGL((fact::wave::k_solve_factored_wave<float, 16>), grid, block, lds, st, metas, plan->n_pixels, x0, pi, infos_dev, o, fact::wave::SpecOut{});
    } else {
      const double* x0 = static_cast<const double*>(x0_packed_dev);
      double* pi = static_cast<double*>(pi_packed_dev);
      if (E == 4) hipLaunchKernelGGL((fact::wave::k_solve_factored_wave<double, 4>), grid, block, lds, st, metas, plan->n_pixels, x0, pi, infos_dev, o, fact::wave::SpecOut{});
      else if (E == 8) hipLaunchKernelGGL((fact::wave::k_solve_factored_wave<double, 8>), grid, block, lds, st, metas, plan->n_pixels, x0, pi, infos_dev, o, fact::wave::SpecOut{});
      else hipLaunchKernelGGL((fact::wave::k_solve_factored_wave<double, 16>), grid, block, lds, st, metas, plan->n_pixels, x0, pi, infos_dev, o, fact::wave::SpecOut{});
    }
    return hipGetLastError() == hipSuccess ? DTM_OK : DTM_EHIP;
  }
  const bool in_lds = plan->max_n <= fact::kLdsMaxN;
  const size_t lds = in_lds ? 5 * sizeof(double) * static_cast<size_t>(plan->max_n) : 0;
  const dim3 grid(plan->n_pixels), block(fact::BT);
  if (plan->dt == DTM_F32) {
    const float* x0 = static_cast<const float*>(x0_packed_dev);
    float* pi = static_cast<float*>(pi_packed_dev);
    if (in_lds) {
      if (hipFuncSetAttribute(reinterpret_cast<const void*>(fact::k_solve_factored<float, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        return DTM_EHIP;
      hipLaunchKernelGGL((fact::k_solve_factored<float, true>), grid, block, lds, st, metas, fact,
                         plan->vec_elems, x0, pi, infos_dev, o);
    } else {
      hipLaunchKernelGGL((fact::k_solve_factored<float, false>), grid, block, 0, st, metas, fact,
                         plan->vec_elems, x0, pi, infos_dev, o);
    }
  } else {
    const double* x0 = static_cast<const double*>(x0_packed_dev);
    double* pi = static_cast<double*>(pi_packed_dev);
    if (in_lds) {
      if (hipFuncSetAttribute(reinterpret_cast<const void*>(fact::k_solve_factored<double, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        return DTM_EHIP;
      hipLaunchKernelGGL((fact::k_solve_factored<double, true>), grid, block, lds, st, metas, fact,
                         plan->vec_elems, x0, pi, infos_dev, o);
    } else {
      hipLaunchKernelGGL((fact::k_solve_factored<double, false>), grid, block, 0, st, metas, fact,
                         plan->vec_elems, x0, pi, infos_dev, o);
    }
  }
  return hipGetLastError() == hipSuccess ? DTM_OK : DTM_EHIP;
}

size_t dtm_spectral_scratch_bytes(const dtm_plan* plan, int32_t with_mixing) {
  if (!plan) return 0;
  // NVEC float64 vectors per pixel for the subspace iteration, c per pixel, and
  // for the mixing search of plans with n above 1024 (one thread per start
  // state) two n x n float64 blocks per pixel plus their offsets; up to
  // 1024 bins the search keeps every start state on chip
  size_t b = align256(8 * fact::NVEC * static_cast<size_t>(plan->vec_elems));
  b += align256(8 * static_cast<size_t>(plan->n_pixels));
  if (with_mixing && plan->max_n > 1024) {
    size_t mix = 0;
    for (const PixelMeta& m : plan->meta) mix += 2 * static_cast<size_t>(m.n) * m.n;
    b += align256(8 * mix) + align256(8 * static_cast<size_t>(plan->n_pixels));
  }
  return b;
}

int dtm_spectral_batched(const dtm_plan* plan, double mixing_eps, int32_t max_steps,
                         dtm_spectral_info* out_dev, void* scratch_dev, size_t scratch_bytes,
                         dtm_stream_t stream) {
  if (!plan || !plan->ws || !out_dev || !scratch_dev || max_steps < 1 || max_steps > (1 << 30))
    return DTM_EINVAL;
  const bool with_mix = mixing_eps > 0.0;
  if (scratch_bytes < dtm_spectral_scratch_bytes(plan, with_mix ? 1 : 0)) return DTM_ENOSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(plan->ws);
  const PixelMeta* metas = reinterpret_cast<const PixelMeta*>(w + plan->off_meta);
  char* s = static_cast<char*>(scratch_dev);
  double* fact = reinterpret_cast<double*>(s);
  size_t off = align256(8 * fact::NVEC * static_cast<size_t>(plan->vec_elems));
  double* scal = reinterpret_cast<double*>(s + off);
  off += align256(8 * static_cast<size_t>(plan->n_pixels));
  KOpts o = plan->kopts;
  o.tol = 1e-13;
  o.safety = 1.0;
  o.stop_rule = DTM_STOP_BOUND;
  o.pad = 0;
  if (with_mix && static_cast<double>(plan->n_pixels) * ((plan->max_n + 3) / 4) >= 2147483647.0)
    return DTM_EINVAL;
  if (plan->max_n <= 1024) {
    // tables and pi by the factored solver's wavefront kernel (one
    // wavefront per pixel, E bins per lane), which then writes them to the
    // scratch instead of returning pi
    const int E = plan->max_n <= 256 ? 4 : plan->max_n <= 512 ? 8 : 16;
    const dim3 grid((plan->n_pixels + 3) / 4), block(fact::BT);
    const size_t lds = sizeof(double) * 4 * 2 * kWave * (E + 1);
    const fact::wave::SpecOut so{fact, plan->vec_elems, scal, out_dev};
    const void* kern = E == 4 ? reinterpret_cast<const void*>(fact::wave::k_solve_factored_wave<double, 4, true>)
                       : E == 8 ? reinterpret_cast<const void*>(fact::wave::k_solve_factored_wave<double, 8, true>)
                                : reinterpret_cast<const void*>(fact::wave::k_solve_factored_wave<double, 16, true>);
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
      return DTM_EHIP;
    if (E == 4)
      hipLaunchKernelGGL((fact::wave::k_solve_factored_wave<double, 4, true>), grid, block, lds, st, metas,
                         plan->n_pixels, static_cast<const double*>(nullptr), static_cast<double*>(nullptr),
                         static_cast<dtm_solve_info*>(nullptr), o, so);
    else if (E == 8)
      hipLaunchKernelGGL((fact::wave::k_solve_factored_wave<double, 8, true>), grid, block, lds, st, metas,
                         plan->n_pixels, static_cast<const double*>(nullptr), static_cast<double*>(nullptr),
                         static_cast<dtm_solve_info*>(nullptr), o, so);
    else
      hipLaunchKernelGGL((fact::wave::k_solve_factored_wave<double, 16, true>), grid, block, lds, st, metas,
                         plan->n_pixels, static_cast<const double*>(nullptr), static_cast<double*>(nullptr),
                         static_cast<dtm_solve_info*>(nullptr), o, so);
  } else {
    hipLaunchKernelGGL(fact::k_spectral_pi, dim3(plan->n_pixels), dim3(fact::BT), 0, st, metas, fact,
                       plan->vec_elems, scal, out_dev, o);
  }
  if (hipGetLastError() != hipSuccess) return DTM_EHIP;
  // the lambda_2 search on the caller's stream and the mixing search on the
  // plan's second stream, side by side (the search keeps one workgroup per
  // pixel busy for its whole run; the mixing workgroups fill the rest)
  hipStream_t mst = st;
  if (with_mix) {
    mst = static_cast<hipStream_t>(plan->aux_stream);
    if (hipEventRecord(static_cast<hipEvent_t>(plan->ev_fork), st) != hipSuccess ||
        hipStreamWaitEvent(mst, static_cast<hipEvent_t>(plan->ev_fork), 0) != hipSuccess)
      return DTM_EHIP;
  }
  if (plan->max_n <= fact::kSpecLdsMaxN) {
    // 15 vectors of 1024 bins (120 KB) leave room on the CU for a
    // workgroup of the mixing search running beside it
    const size_t lds = fact::NVEC_LDS * sizeof(double) * static_cast<size_t>(plan->max_n);
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(fact::k_spectral<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
      return DTM_EHIP;
    hipLaunchKernelGGL(fact::k_spectral<true>, dim3(plan->n_pixels), dim3(fact::BT), lds, st, metas, fact,
                       plan->vec_elems, scal, out_dev, max_steps);
  } else {
    hipLaunchKernelGGL(fact::k_spectral<false>, dim3(plan->n_pixels), dim3(fact::BT), 0, st, metas, fact,
                       plan->vec_elems, scal, out_dev, max_steps);
  }
  if (hipGetLastError() != hipSuccess) return DTM_EHIP;
  if (!with_mix) return DTM_OK;
  const auto join = [&]() {
    if (hipEventRecord(static_cast<hipEvent_t>(plan->ev_join), mst) != hipSuccess ||
        hipStreamWaitEvent(st, static_cast<hipEvent_t>(plan->ev_join), 0) != hipSuccess)
      return DTM_EHIP;
    return DTM_OK;
  };
  if (plan->max_n <= 1024) {
    // one wavefront per start state, four per block; E bins per lane
    const int E = plan->max_n <= 256 ? 4 : plan->max_n <= 512 ? 8 : 16;
    const int sb = (plan->max_n + 3) / 4;
    const dim3 grid(static_cast<unsigned>(plan->n_pixels) * static_cast<unsigned>(sb));
    const size_t lds = sizeof(double) * 4 * kWave * (E + 1);
    if (E == 4)
      hipLaunchKernelGGL(fact::k_mixing_wave<4>, grid, dim3(fact::BT), lds, mst, metas, fact, plan->vec_elems, scal,
                         out_dev, mixing_eps, max_steps, sb);
    else if (E == 8)
      hipLaunchKernelGGL(fact::k_mixing_wave<8>, grid, dim3(fact::BT), lds, mst, metas, fact, plan->vec_elems, scal,
                         out_dev, mixing_eps, max_steps, sb);
    else
      hipLaunchKernelGGL(fact::k_mixing_wave<16>, grid, dim3(fact::BT), lds, mst, metas, fact, plan->vec_elems,
                         scal, out_dev, mixing_eps, max_steps, sb);
    if (hipGetLastError() != hipSuccess) return DTM_EHIP;
    hipLaunchKernelGGL(fact::k_mixing_final, dim3((plan->n_pixels + fact::BT - 1) / fact::BT), dim3(fact::BT), 0,
                       mst, metas, plan->n_pixels, out_dev, max_steps);
    if (hipGetLastError() != hipSuccess) return DTM_EHIP;
    return join();
  }
  // larger pixels: the n x n blocks of start-state distributions live in the
  // scratch, at per-pixel offsets copied from the host
  std::vector<int64_t> offs(plan->n_pixels);
  size_t mix = 0;
  for (int32_t q = 0; q < plan->n_pixels; ++q) {
    offs[q] = static_cast<int64_t>(mix);
    mix += 2 * static_cast<size_t>(plan->meta[q].n) * plan->meta[q].n;
  }
  double* mixbuf = reinterpret_cast<double*>(s + off);
  off += align256(8 * mix);
  int64_t* mix_off = reinterpret_cast<int64_t*>(s + off);
  if (hipMemcpyAsync(mix_off, offs.data(), sizeof(int64_t) * offs.size(), hipMemcpyHostToDevice, mst) !=
      hipSuccess)
    return DTM_EHIP;
  {
    const int sb = (plan->max_n + fact::BT - 1) / fact::BT;
    hipLaunchKernelGGL(fact::k_mixing, dim3(static_cast<unsigned>(plan->n_pixels) * static_cast<unsigned>(sb)),
                       dim3(fact::BT), 0, mst, metas, fact, plan->vec_elems, mixbuf, mix_off, scal, out_dev,
                       mixing_eps, max_steps, sb);
  }
  if (hipGetLastError() != hipSuccess) return DTM_EHIP;
  hipLaunchKernelGGL(fact::k_mixing_final, dim3((plan->n_pixels + fact::BT - 1) / fact::BT), dim3(fact::BT), 0, mst,
                     metas, plan->n_pixels, out_dev, max_steps);
  if (hipGetLastError() != hipSuccess) return DTM_EHIP;
  const int rc = join();
  if (rc) return rc;
  // the offsets must outlive the asynchronous copy
  if (hipStreamSynchronize(st) != hipSuccess) return DTM_EHIP;
  return DTM_OK;
}

}  // extern "C"
