// Device building blocks for gfx950: reductions, bin tables, row sums and
// the per-element value of the transition matrix.
#pragma once

#include <hip/hip_runtime.h>

#include "dtm_internal.h"

namespace dtm {

constexpr int kWave = 64;

template <typename T>
struct Vec;
template <>
struct Vec<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};
template <>
struct Vec<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};

// ---- reductions (fixed order: results are bitwise reproducible) ----------

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sums of a, b and c over the block; every thread gets all three.  `red` is
// LDS with room for 3 * BT / 64 doubles.
template <int BT>
__device__ inline void block_sum3(double& a, double& b, double& c, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  constexpr int NW = BT / kWave;
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x % kWave) == 0) {
    red[w] = a;
    red[NW + w] = b;
    red[2 * NW + w] = c;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0, sc = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    sa += red[i];
    sb += red[NW + i];
    sc += red[2 * NW + i];
  }
  a = sa;
  b = sb;
  c = sc;
}

template <int BT>
__device__ inline void block_sum2(double& a, double& b, double* red) {
  double c = 0.0;
  block_sum3<BT>(a, b, c, red);
}

template <int BT>
__device__ inline double block_sum(double a, double* red) {
  double b = 0.0, c = 0.0;
  block_sum3<BT>(a, b, c, red);
  return a;
}

// Exclusive prefix sum over the block in thread order; `total` gets the sum.
template <int BT>
__device__ inline double block_exclusive_scan(double v, double* red, double& total) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  double x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const double y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  double excl = __shfl_up(x, 1, kWave);
  if (lane == 0) excl = 0.0;
  __syncthreads();
  if (lane == kWave - 1) red[w] = x;
  __syncthreads();
  double base = 0.0, tot = 0.0;
#pragma unroll
  for (int i = 0; i < BT / kWave; ++i) {
    if (i < w) base += red[i];
    tot += red[i];
  }
  total = tot;
  return base + excl;
}

// Exclusive prefix sum in reversed thread order: thread t gets the sum of v
// over threads t+1 .. BT-1.
template <int BT>
__device__ inline double block_exclusive_scan_rev(double v, double* red) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  double x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const double y = __shfl_down(x, off, kWave);
    if (lane + off < kWave) x += y;
  }
  double excl = __shfl_down(x, 1, kWave);
  if (lane == kWave - 1) excl = 0.0;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double base = 0.0;
#pragma unroll
  for (int i = BT / kWave - 1; i >= 0; --i)
    if (i > w) base += red[i];
  return base + excl;
}

// Compensated (Kahan) accumulation; the sum is s - c.  float64 needs none.
__device__ inline void comp_add(float& s, float& c, float v) {
  const float y = v - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}
__device__ inline void comp_add(double& s, double& c, double v) {
  (void)c;
  s += v;
}

// ---- bin tables ------------------------------------------------------------

// Normal tail beyond z on z's side: 1 - Phi(z) for z >= 0, Phi(z) for z < 0.
__device__ inline double gauss_tail(double z) {
  return 0.5 * erfc(fabs(z) * 0.70710678118654752440);
}

// Normal mass on [za, zb] (za <= zb) from the tails at its ends (gauss_tail),
// each difference taken where it keeps its digits.
__device__ inline double mass_from_tails(double za, double ta, double zb, double tb) {
  if (za >= 0.0) return ta - tb;
  if (zb <= 0.0) return tb - ta;
  return 1.0 - ta - tb;
}

// lambda(t) = S N(t - tau; 0, sigma^2) + B / t_r (Eq. arrival_flux).
__device__ inline double flux_at(const PixelMeta& m, double t) {
  const double z = (t - m.tau) / m.sigma;
  return m.S * exp(-0.5 * z * z) * (0.39894228040143267794 / m.sigma) + m.B / m.t_r;
}

// Bin tables of one pixel, computed by the whole block (BT threads).
// F_j = F(s_j) (Theorem 1) is an exclusive float64 prefix sum of per-bin
// integrals plus the half-bin integral up to the centre; Lambda = F(t_r).
// Writes g_j = lambda_j exp(-F_j) in T for j < n and 0 for n <= j < ld
// (g may point to LDS or global memory), and optionally lambda_j (T) and
// F_j (float64, with F_n = Lambda).  Returns Lambda.
template <typename T, int BT>
__device__ double pixel_tables(const PixelMeta& m, T* g, T* lam_out, double* F_out, double* red) {
  const int n = m.n;
  const double delta = m.t_r / n;
  const int chunk = (n + BT - 1) / BT;
  const int j0 = min(static_cast<int>(threadIdx.x) * chunk, n);
  const int j1 = min(j0 + chunk, n);
  // Normal tails at the bin edges and centres: one erfc per edge and one per
  // centre (an edge is shared by two bins; a chunk's total needs only its
  // two end edges).
  const double is = 1.0 / m.sigma;
  const double bq = m.B / m.t_r;
  const double z0 = (j0 * delta - m.tau) * is, z1 = (j1 * delta - m.tau) * is;
  double part = 0.0;
  if (j1 > j0)
    part = m.S * mass_from_tails(z0, gauss_tail(z0), z1, gauss_tail(z1)) + bq * ((j1 - j0) * delta);
  double total;
  double acc = block_exclusive_scan<BT>(part, red, total);
  double zl = z0, tl = gauss_tail(z0);
  for (int j = j0; j < j1; ++j) {
    const double lo = j * delta;
    const double zm = (lo + 0.5 * delta - m.tau) * is, zh = ((j + 1) * delta - m.tau) * is;
    const double tm = gauss_tail(zm), th = gauss_tail(zh);
    const double F = acc + m.S * mass_from_tails(zl, tl, zm, tm) + bq * (0.5 * delta);
    const double dF = m.S * mass_from_tails(zl, tl, zh, th) + bq * delta;
    zl = zh;
    tl = th;
    double lj, gj;
    if (m.lam_mode == 0) {  // lambda at the bin centre (Section 3.4)
      lj = flux_at(m, lo + 0.5 * delta);
      gj = lj * exp(-F);
    } else if (m.lam_mode == 1) {  // lambda averaged over the bin
      lj = dF / delta;
      gj = lj * exp(-F);
    } else {  // lambda e^{-F} averaged over the bin: (e^{-F(lo)} - e^{-F(hi)}) / Delta
      gj = exp(-acc) * -expm1(-dF) / delta;
      lj = gj * exp(F);
    }
    acc += dF;
    g[j] = static_cast<T>(gj);
    if (lam_out) lam_out[j] = static_cast<T>(lj);
    if (F_out) F_out[j] = F;
  }
  for (int j = n + threadIdx.x; j < m.ld; j += BT) g[j] = T(0);
  if (F_out && threadIdx.x == 0) F_out[n] = total;
  return total;
}

// Row normalisers of the base matrix (Section 3.4).  Row k of E_base times
// lambda is exp(F_k) * g_j * w_kj with w_kj = c = exp(-Lambda) for j < k (the
// wrap term of Theorem 1's indicator) and 1 otherwise; the common factor
// exp(F_k) cancels in the normalisation, leaving
//   S_k = sum_j g_j w_kj = sum_{j >= k} g_j + c * sum_{j < k} g_j.
// Every row holds the same g and differs only in where the wrap factor
// starts, so one prefix and one suffix float64 block scan give all n row sums
// with no subtraction.  The block owns chunks of bins exactly as in
// pixel_tables (so each thread reads only g values it wrote itself); pk is
// float64 scratch of n entries.  Writes invs[k] = 1 / S_k.
template <typename T, int BT>
__device__ void row_normalisers(int n, const T* g, T c, double* pk, T* invs, double* red) {
  const int chunk = (n + BT - 1) / BT;
  const int j0 = min(static_cast<int>(threadIdx.x) * chunk, n);
  const int j1 = min(j0 + chunk, n);
  const double cd = static_cast<double>(c);
  double cs = 0.0;
  for (int j = j0; j < j1; ++j) cs += static_cast<double>(g[j]);
  double tot;
  const double pre = block_exclusive_scan<BT>(cs, red, tot);
  const double suf = block_exclusive_scan_rev<BT>(cs, red);
  double P = pre;
  for (int j = j0; j < j1; ++j) {
    pk[j] = P;
    P += static_cast<double>(g[j]);
  }
  double Tk = suf;
  for (int j = j1 - 1; j >= j0; --j) {
    Tk += static_cast<double>(g[j]);
    invs[j] = static_cast<T>(1.0 / (Tk + cd * pk[j]));
  }
}

// Row sum S_k = sum_j g_j w_kj with w_kj = c for j < k (the wrap term
// exp(-Lambda) of Theorem 1's indicator) and 1 otherwise, by one wavefront:
// per-lane compensated partials, then a float64 butterfly.  The row factor
// exp(F_k) of E is common to the whole row and cancels in the normalisation,
// so it is never formed.  Returns the sum on every lane.
template <typename T>
__device__ inline double wave_row_sum(const T* g, int n, int k, T c) {
  const int lane = threadIdx.x % kWave;
  T s = T(0), comp = T(0);
  for (int j = lane; j < n; j += kWave) {
    const T v = g[j] * (j < k ? c : T(1));
    comp_add(s, comp, v);
  }
  return wave_sum(static_cast<double>(s) - static_cast<double>(comp));
}

// ============================================================================
// Stop rule.  The error of power iteration decays like |lambda_2|^t
// (Section 4); its phase decides whether the iterates approach pi
// monotonically or oscillate around it.  After sweep t with difference
// vector d_t = x_{t+1} - x_t:
//   rho  = max(c_t / c_{t-1}, sqrt(c_t / c_{t-2}))     (|lambda_2| estimate)
//   if d_t is parallel to d_{t-1} (a real dominant eigenvalue mu, estimated
//   by projection), the remaining error is |mu| / (1 - mu) * ||d_t||, which
//   is small for an alternating mu < 0; otherwise the phase-free worst case
//   rho / (1 - rho) is used.
// Every thread of a block runs this on identical inputs.
// ============================================================================

__device__ inline void stop_init(StopState& s, int warm, int flags) {
  s.c1 = s.c2 = s.c3 = 0.0;
  s.rho = 0.999;
  s.gain = 999.0;
  s.contr = 0.999;
  s.resid = 0.0;
  s.dd_prev = 0.0;
  s.iter = 0;
  s.total_iter = 0;
  s.check_next = 0;
  s.done = 0;
  s.status = DTM_OK;
  s.flags = flags;
  s.warm = warm;
  s.stalled = 0;
}

__device__ inline double estimate_rho(double c1, double c2, double c3, int t) {
  double rho;
  if (t <= 1 || !(c2 > 0.0)) {
    rho = (t <= 1) ? 0.999 : 0.0;
  } else {
    rho = c1 / c2;
    if (t >= 3 && c3 > 0.0) rho = fmax(rho, sqrt(c1 / c3));
  }
  return fmin(fmax(rho, 0.0), 0.999);
}

// Updates the state after a sweep: change = ||d_t||_1, dd = ||d_t||_2^2,
// ddp = <d_t, d_{t-1}>, resid = ||x_t P - x_t||_1 (float64 on a check
// sweep), eps = unit round-off of the iterate's type.  Returns true when the
// caller must restart from the uniform vector (a warm start that failed).
__device__ inline bool stop_update(StopState& s, const KOpts& o, double change, double dd,
                                   double ddp, double resid, bool was_check, double eps) {
  s.iter += 1;
  s.total_iter += 1;
  s.c3 = s.c2;
  s.c2 = s.c1;
  s.c1 = change;
  // Ratios of changes near the round-off floor are noise: keep the last
  // estimate made above 64 units of round-off.
  if (s.iter <= 2 || change >= 64.0 * eps) {
    s.rho = estimate_rho(s.c1, s.c2, s.c3, s.iter);
    double g = s.rho / (1.0 - s.rho), k = s.rho;
    if (s.iter >= 2 && s.dd_prev > 0.0 && dd > 0.0) {
      const double mu = ddp / s.dd_prev;
      const double cos2 = (ddp * ddp) / (dd * s.dd_prev);
      if (cos2 >= 0.99 && mu < 0.999 && fabs(mu) / (1.0 - mu) < g) {
        g = fabs(mu) / (1.0 - mu);
        k = fabs(mu);
      }
    }
    s.gain = g;
    s.contr = k;
  }
  const double gain = s.gain;
  s.dd_prev = dd;
  // No progress over two sweeps at the round-off floor of the iterate.
  const bool stalled = s.iter >= 3 && change > 0.0 && change >= s.c3 && change < 4096.0 * eps;
  if (stalled) s.stalled = 1;
  s.resid = resid;
  if (was_check) {
    s.flags |= DTM_INFO_CHECKED;
    const bool ok = (o.stop_rule == DTM_STOP_CHANGE) ? (change < o.tol)
                                                     : (resid * gain <= o.safety * o.tol);
    if (ok) {
      s.done = 1;
      s.status = DTM_OK;
      return false;
    }
    if (s.stalled) {  // cannot improve further in this precision
      s.flags |= DTM_INFO_STALLED;
      s.done = 1;
      s.status = DTM_ENOTCONV;
      return false;
    }
    s.check_next = 0;
  } else {
    // The check sweep's residual will be about the next change, contr times
    // this one: fire when that one is predicted to pass.  A check that fails
    // costs nothing extra (its output is the next iterate), and the check
    // never comes later than when this change itself passes.  Without a
    // check the iterate at hand is the answer, so this change must pass.
    const double ahead = o.final_check ? s.contr : 1.0;
    const bool fire = (o.stop_rule == DTM_STOP_CHANGE)
                          ? (change < o.tol)
                          : (change == 0.0 || (s.iter >= 2 && change * gain * ahead <= o.safety * o.tol));
    if (fire || s.stalled) {
      if (o.final_check) {
        s.check_next = 1;
      } else if (fire) {
        s.done = 1;
        s.status = DTM_OK;
        return false;
      } else {
        s.flags |= DTM_INFO_STALLED;
        s.done = 1;
        s.status = DTM_ENOTCONV;
        return false;
      }
    }
  }
  if (s.iter >= o.max_iter) {
    if (s.warm && !(s.flags & DTM_INFO_RESTARTED)) {
      s.flags |= DTM_INFO_RESTARTED;
      s.iter = 0;
      s.c1 = s.c2 = s.c3 = 0.0;
      s.dd_prev = 0.0;
      s.check_next = 0;
      s.stalled = 0;
      return true;
    }
    s.done = 1;
    s.status = DTM_ENOTCONV;
  }
  return false;
}

__device__ inline dtm_solve_info make_info(const StopState& s) {
  dtm_solve_info info;
  info.iterations = s.total_iter;
  info.status = s.status;
  info.flags = s.flags;
  info.dense_sweeps = s.total_iter;
  info.change_l1 = s.c1;
  info.residual_l1 = s.resid;
  info.rho_hat = s.rho;
  return info;
}

}  // namespace dtm
