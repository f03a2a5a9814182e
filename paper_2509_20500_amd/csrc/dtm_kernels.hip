// HIP kernels for gfx950 and the C-ABI entry points that launch them.
//
// Matrix element (Section 3.4, Eq. Eij_ours with the row permutation J_l):
//   P~[i, j] = lambda_j exp(-Lambda [k > j] - F_j + F_k) / R_k,  k = (i + l) mod n
//            = g_j w_kj / S_k,   g_j = lambda_j exp(-F_j),  w_kj = exp(-Lambda) if j < k else 1,
// where S_k = sum_j g_j w_kj is the row sum of the base matrix with its common
// row factor exp(F_k) cancelled.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "dtm_device.hpp"
#include "dtm_internal.h"

namespace dtm {

// ============================================================================
// Kernels shared by the single-pixel and the batched entry points.  A launch
// covers `metas[0 .. gridDim.y)` (device array) or the single pixel `one`
// when metas is null.
// ============================================================================

template <typename V>
__device__ inline V zero_vec() {
  V v;
#pragma unroll
  for (int e = 0; e < static_cast<int>(sizeof(V) / sizeof(v[0])); ++e) v[e] = 0;
  return v;
}

__device__ inline PixelMeta load_meta(const PixelMeta* metas, const PixelMeta& one, int p) {
  return metas ? metas[p] : one;
}

// Bin tables: one block per pixel.  g -> colf[vec_off ...], c = exp(-Lambda)
// -> scal[p]; lambda and F to the caller's buffers when given.
// Bin tables and row normalisers: one block per pixel.  g -> colf[vec_off],
// 1/S_k -> invs[vec_off], c = exp(-Lambda) -> scal[p] (pk: float64 scratch
// with the layout of colf); lambda and F to the caller's buffers when given.
template <typename T, int BT>
__global__ __launch_bounds__(BT) void k_tables(const PixelMeta* metas, PixelMeta one, T* colf,
                                               T* invs, double* pk, double* scal, T* lam_out,
                                               double* F_out) {
  __shared__ double red[3 * BT / kWave];
  const PixelMeta m = load_meta(metas, one, blockIdx.x);
  const double Lam = pixel_tables<T, BT>(m, colf + m.vec_off, lam_out, F_out, red);
  const double c = exp(-Lam);
  row_normalisers<T, BT>(m.n, colf + m.vec_off, static_cast<T>(c), pk + m.vec_off,
                         invs + m.vec_off, red);
  if (threadIdx.x == 0) scal[blockIdx.x] = c;
}

// Writes rows of the transition matrix, one wavefront per row, lanes over
// columns in 16-byte vectors.  shifted: row i is built from base row
// (i + l) mod n (Theorem 2); otherwise from row i.  Output element (i, j) of
// pixel p is at out + base + i * ld + j with base/ld either the padded pool
// layout (packed = 0) or the caller's packed layout (packed = 1, ld = n).
template <typename T, int BT, int ROWS_PER_WAVE>
__global__ __launch_bounds__(BT) void k_build(const PixelMeta* metas, PixelMeta one, const T* colf,
                                              const double* scal, const T* invs, T* out,
                                              int64_t out_ld_single, int shifted, int packed) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  const PixelMeta m = load_meta(metas, one, blockIdx.y);
  const int n = m.n;
  const int64_t ld = metas ? (packed ? m.n : m.ld) : out_ld_single;
  const int64_t base = metas ? (packed ? m.out_off : m.mat_off) : 0;
  const T c = static_cast<T>(scal[blockIdx.y]);
  const T* g = colf + m.vec_off;
  const int lane = threadIdx.x % kWave;
  const int wave = blockIdx.x * (BT / kWave) + threadIdx.x / kWave;
  const bool vec_ok = (ld % VN == 0) && (base % VN == 0) &&
                      ((reinterpret_cast<uintptr_t>(out) % 16) == 0);
  const bool pool_layout = metas && !packed;  // rows padded to ld, padding owned by the library
  for (int r = 0; r < ROWS_PER_WAVE; ++r) {
    const int i = wave * ROWS_PER_WAVE + r;
    if (i >= n) return;
    int k = i;
    if (shifted) {
      k = i + m.l;
      if (k >= n) k -= n;
    }
    const T s = invs[m.vec_off + k];
    T* row = out + base + static_cast<int64_t>(i) * ld;
    if (vec_ok) {
      for (int j0 = lane * VN; j0 < n; j0 += kWave * VN) {
        const V gv = *reinterpret_cast<const V*>(g + j0);  // g is zero-padded to ld
        V v;
#pragma unroll
        for (int e = 0; e < VN; ++e) v[e] = gv[e] * ((j0 + e) < k ? c : T(1)) * s;
        if (j0 + VN <= n || pool_layout) {
          *reinterpret_cast<V*>(row + j0) = v;
        } else {
#pragma unroll
          for (int e = 0; e < VN; ++e)
            if (j0 + e < n) row[j0 + e] = v[e];
        }
      }
    } else {
      for (int j = lane; j < n; j += kWave) row[j] = g[j] * (j < k ? c : T(1)) * s;
    }
  }
}

// Dead time as a row permutation (Theorem 2): dst[i, :] = src[(i + l) mod n, :].
template <typename T, int BT, int ROWS_PER_WAVE>
__global__ __launch_bounds__(BT) void k_shift(const PixelMeta* metas, PixelMeta one, const T* src,
                                              T* dst, int64_t ld_single) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  const PixelMeta m = load_meta(metas, one, blockIdx.y);
  const int n = m.n;
  const int64_t ld = metas ? m.n : ld_single;
  const int64_t base = metas ? m.out_off : 0;
  const int lane = threadIdx.x % kWave;
  const int wave = blockIdx.x * (BT / kWave) + threadIdx.x / kWave;
  const bool vec_ok = (ld % VN == 0) && (base % VN == 0) &&
                      ((reinterpret_cast<uintptr_t>(src) % 16) == 0) &&
                      ((reinterpret_cast<uintptr_t>(dst) % 16) == 0);
  for (int r = 0; r < ROWS_PER_WAVE; ++r) {
    const int i = wave * ROWS_PER_WAVE + r;
    if (i >= n) return;
    int k = i + m.l;
    if (k >= n) k -= n;
    const T* a = src + base + static_cast<int64_t>(k) * ld;
    T* b = dst + base + static_cast<int64_t>(i) * ld;
    if (vec_ok) {
      const int nv = n / VN;
      for (int q = lane; q < nv; q += kWave)
        reinterpret_cast<V*>(b)[q] = reinterpret_cast<const V*>(a)[q];
      for (int j = nv * VN + lane; j < n; j += kWave) b[j] = a[j];
    } else {
      for (int j = lane; j < n; j += kWave) b[j] = a[j];
    }
  }
}

// ============================================================================
// Batched solver for pixels that fit one block: per pixel, the shifted build
// with the first power-iteration sweep taken on the way, the remaining
// sweeps, the float64 check sweep and the stop rule.  The bin tables g_j,
// 1/S_k and c = exp(-Lambda) come from k_tables (run just before, so that its
// erf code does not set these kernels' register budgets).  Thread t owns columns
// (t + BT q) * VN .. + VN - 1 for q < CPT in every row: each row is one
// coalesced pass of the block and x P~ needs no cross-thread reduction.
// ============================================================================

template <typename V>
__device__ inline V stream_load(const V* p) {
#if DTM_NT_LOADS
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

// y += x_i P[i, :] over rows [i0, i1) for this thread's columns, UE rows in
// flight plus the next UE rows prefetched.  Addresses of columns past n are
// clamped to column 0 (those lanes' sums are never used), so the loads carry
// no per-lane guards.
template <typename T, int BT, int CPT, int UE, bool CHECK, typename A>
__device__ inline void sweep_rows(const T* __restrict__ mat, int64_t ld, int n, const int* jc,
                                  const T* __restrict__ xs, A (&acc)[CPT][Vec<T>::n],
                                  A (&cmp)[CPT][Vec<T>::n]) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  int i0 = 0;
  if (n >= UE) {
    V cur[UE][CPT];
#pragma unroll
    for (int u = 0; u < UE; ++u)
#pragma unroll
      for (int q = 0; q < CPT; ++q)
        cur[u][q] = stream_load(
            reinterpret_cast<const V*>(mat + static_cast<int64_t>(u) * ld + jc[q]));
    for (; i0 + UE <= n; i0 += UE) {
      V nxt[UE][CPT];
      const bool more = i0 + 2 * UE <= n;
      if (more) {
#pragma unroll
        for (int u = 0; u < UE; ++u)
#pragma unroll
          for (int q = 0; q < CPT; ++q)
            nxt[u][q] = stream_load(reinterpret_cast<const V*>(
                mat + static_cast<int64_t>(i0 + UE + u) * ld + jc[q]));
      }
#pragma unroll
      for (int u = 0; u < UE; ++u) {
        const T xi = xs[i0 + u];
#pragma unroll
        for (int q = 0; q < CPT; ++q)
#pragma unroll
          for (int e = 0; e < VN; ++e) {
            if constexpr (CHECK)
              acc[q][e] += static_cast<double>(xi) * static_cast<double>(cur[u][q][e]);
            else
              comp_add(acc[q][e], cmp[q][e], xi * cur[u][q][e]);
          }
      }
      if (more) {
#pragma unroll
        for (int u = 0; u < UE; ++u)
#pragma unroll
          for (int q = 0; q < CPT; ++q) cur[u][q] = nxt[u][q];
      }
    }
  }
  for (; i0 < n; ++i0) {
    const T xi = xs[i0];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const V v = *reinterpret_cast<const V*>(mat + static_cast<int64_t>(i0) * ld + jc[q]);
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        if constexpr (CHECK)
          acc[q][e] += static_cast<double>(xi) * static_cast<double>(v[e]);
        else
          comp_add(acc[q][e], cmp[q][e], xi * v[e]);
      }
    }
  }
}

// The dense solve of a batch runs in two launches over the same pixels (one
// block each, same order): k_solve_build writes every matrix while it takes
// the first sweep, then k_solve_sweeps runs the remaining sweeps, which only
// read.  Measured on this part, HBM gives a stream of writes followed by a
// stream of reads about 1.3 times the bandwidth it gives the same traffic
// mixed (each block writing its matrix and then reading it back while others
// write theirs).  The first sweep's float64 sums y = x0 P~ pass between the
// launches through the workspace; the start vector is derived again, the
// same way, so the iterates are those of one fused kernel, bit for bit.

// Flux at the centre of bin j, lambda(s_j) = S N(s_j; tau, sigma^2) + B / t_r
// (the model's point sampling; only a start vector is made from it).
__device__ inline double start_flux_value(const PixelMeta& m, int j) {
  const double s = (j + 0.5) * (m.t_r / m.n);
  const double z = (s - m.tau) / m.sigma;
  return m.S * exp(-0.5 * z * z) / (m.sigma * 2.5066282746310002) + m.B / m.t_r;
}

// Start vector into xs (LDS): the caller's, validated and normalised; else
// lambda / sum(lambda) when flux is set; else the uniform one; records the
// warm start in st.  Ends with a block barrier.
template <typename T, int BT>
__device__ inline void start_vector(const PixelMeta& m, const T* __restrict__ x0_packed, int flux, T* xs,
                                    StopState& st, double* red) {
  const int n = m.n, tid = threadIdx.x;
  if (x0_packed) {
    double sum = 0.0, bad = 0.0;
    for (int j = tid; j < n; j += BT) {
      const double v = static_cast<double>(x0_packed[m.pi_off + j]);
      if (!(v >= 0.0) || !isfinite(v)) bad += 1.0;
      else sum += v;
    }
    block_sum2<BT>(sum, bad, red);
    if (bad == 0.0 && sum > 0.0 && isfinite(sum)) {
      st.warm = 1;
      for (int j = tid; j < n; j += BT)
        xs[j] = static_cast<T>(static_cast<double>(x0_packed[m.pi_off + j]) / sum);
    } else {
      st.flags |= DTM_INFO_WARM_REJECTED;
      for (int j = tid; j < n; j += BT) xs[j] = static_cast<T>(1.0 / n);
    }
  } else if (flux) {
    double sum = 0.0, unused = 0.0;
    for (int j = tid; j < n; j += BT) sum += start_flux_value(m, j);
    block_sum2<BT>(sum, unused, red);
    // a flux that underflows at every centre (possible under the bin-averaged
    // variants, whose matrix is still defined) falls back to uniform
    const bool ok = sum > 0.0 && isfinite(sum);
    for (int j = tid; j < n; j += BT)
      xs[j] = ok ? static_cast<T>(start_flux_value(m, j) / sum) : static_cast<T>(1.0 / n);
  } else {
    for (int j = tid; j < n; j += BT) xs[j] = static_cast<T>(1.0 / n);
  }
  __syncthreads();
}

// Phase 1: tables into LDS, then every row written once (a2 + a3: row i from
// base row k = (i + l) mod n) while x0 P~ accumulates in compensated sums;
// the sums go to y1 (float64, the pixel's ld slots at vec_off).
template <typename T, int BT, int CPT>
__global__ __launch_bounds__(BT) void k_solve_build(const PixelMeta* __restrict__ metas,
                                                    const T* __restrict__ colf,
                                                    const T* __restrict__ invs_g,
                                                    const double* __restrict__ scal,
                                                    T* __restrict__ pool,
                                                    const T* __restrict__ x0_packed,
                                                    double* __restrict__ y1,
                                                    const int32_t* __restrict__ sel, int lds_ld,
                                                    int start_flux, int* __restrict__ queue) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  // the persistent sweep launch that follows on this stream takes pixels
  // from this counter
  if (queue && blockIdx.x == 0 && threadIdx.x == 0) *queue = 0;
  extern __shared__ __align__(16) unsigned char smem[];
  T* g = reinterpret_cast<T*>(smem);
  T* xs = g + lds_ld;
  T* invs = xs + lds_ld;
  double* red = reinterpret_cast<double*>(invs + lds_ld);

  const int pq = sel[blockIdx.x];
  const PixelMeta m = metas[pq];
  const int n = m.n;
  const int64_t ld = m.ld;
  const int tid = threadIdx.x;
  T* mat = pool + m.mat_off;
  const T c = static_cast<T>(scal[pq]);

  for (int j = tid; j < m.ld; j += BT) g[j] = colf[m.vec_off + j];
  for (int j = tid; j < n; j += BT) invs[j] = invs_g[m.vec_off + j];
  __syncthreads();
  StopState st;
  stop_init(st, 0, 0);
  start_vector<T, BT>(m, x0_packed, start_flux, xs, st, red);

  T gr[CPT][VN];
  T acc[CPT][VN], cmp[CPT][VN];
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int j0 = (tid + BT * q) * VN;
#pragma unroll
    for (int e = 0; e < VN; ++e) {
      gr[q][e] = (j0 < n) ? g[j0 + e] : T(0);
      acc[q][e] = cmp[q][e] = T(0);
    }
  }
  for (int i = 0; i < n; ++i) {
    int k = i + m.l;
    if (k >= n) k -= n;
    const T s = invs[k];
    const T xi = xs[i];
    T* row = mat + static_cast<int64_t>(i) * ld;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int j0 = (tid + BT * q) * VN;
      V v;
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        v[e] = gr[q][e] * ((j0 + e) < k ? c : T(1)) * s;
        comp_add(acc[q][e], cmp[q][e], xi * v[e]);
      }
      if (j0 < n) __builtin_nontemporal_store(v, reinterpret_cast<V*>(row + j0));
    }
  }
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int j0 = (tid + BT * q) * VN;
#pragma unroll
    for (int e = 0; e < VN; ++e)
      if (j0 + e < n) y1[m.vec_off + j0 + e] = static_cast<double>(acc[q][e]) - static_cast<double>(cmp[q][e]);
  }
}

// Phase 2: from y1, the stop rule and the remaining sweeps (a4, with the
// float64 check sweep of a5 when due), reading each matrix as many times as
// its pixel needs.
template <typename T, int BT, int CPT, int U>
__global__ __launch_bounds__(BT) void k_solve_sweeps(const PixelMeta* __restrict__ metas,
                                                     const T* __restrict__ pool,
                                                     const T* __restrict__ x0_packed,
                                                     const double* __restrict__ y1,
                                                     T* __restrict__ pi_packed,
                                                     dtm_solve_info* __restrict__ infos,
                                                     const int32_t* __restrict__ sel,
                                                     KOpts o, int lds_ld, int dense_cap,
                                                     T* __restrict__ xbuf,
                                                     SolveState* __restrict__ states,
                                                     int* __restrict__ queue, int count) {
  constexpr int VN = Vec<T>::n;
  constexpr int UE = (U * CPT <= 8) ? U : (8 / CPT > 0 ? 8 / CPT : 1);
  extern __shared__ __align__(16) unsigned char smem[];
  T* xs = reinterpret_cast<T*>(smem);
  double* red = reinterpret_cast<double*>(xs + lds_ld);
  __shared__ int next_pixel;

  // one pixel from its first-sweep sums to its stop (or its dense budget)
  const auto solve = [&](const int pq) {
  const PixelMeta m = metas[pq];
  const int n = m.n;
  const int64_t ld = m.ld;
  const int tid = threadIdx.x;
  const T* mat = pool + m.mat_off;

  StopState st;
  stop_init(st, 0, 0);
  start_vector<T, BT>(m, x0_packed, o.start_flux, xs, st, red);

  // This thread's columns (clamped to 0 past n: those sums are never used).
  int jc[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int j0 = (tid + BT * q) * VN;
    jc[q] = j0 < n ? j0 : 0;
  }

  T acc[CPT][VN], cmp[CPT][VN];
  double accd[CPT][VN], dd0[CPT][VN];
  double dprev[CPT][VN];  // previous difference vector on this thread's columns
#pragma unroll
  for (int q = 0; q < CPT; ++q)
#pragma unroll
    for (int e = 0; e < VN; ++e) {
      dprev[q][e] = 0.0;
      acc[q][e] = cmp[q][e] = T(0);
    }
  bool first = true;        // y is the first sweep's, from phase 1
  bool have_check = false;  // the accumulators hold a float64 check sweep

  for (;;) {
    // ---- reduce: sum of y = x P~, residual ||y - x||_1, then the new
    //      iterate y / sum(y) and its change ------------------------------
    double y[CPT][VN];
    double sy = 0.0, rs = 0.0;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int j0 = (tid + BT * q) * VN;
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        if (first) y[q][e] = (j0 + e < n) ? y1[m.vec_off + j0 + e] : 0.0;
        else
          y[q][e] = have_check ? accd[q][e]
                               : static_cast<double>(acc[q][e]) - static_cast<double>(cmp[q][e]);
        if (j0 + e < n) {
          sy += y[q][e];
          rs += fabs(y[q][e] - static_cast<double>(xs[j0 + e]));
        }
      }
    }
    first = false;
    block_sum2<BT>(sy, rs, red);
    const double inv = 1.0 / sy;
    T xn[CPT][VN];
    double ch = 0.0, dd = 0.0, ddp = 0.0;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int j0 = (tid + BT * q) * VN;
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        xn[q][e] = static_cast<T>(y[q][e] * inv);
        const double dj = (j0 + e < n)
                              ? static_cast<double>(xn[q][e]) - static_cast<double>(xs[j0 + e])
                              : 0.0;
        ch += fabs(dj);
        dd += dj * dj;
        ddp += dj * dprev[q][e];
        dprev[q][e] = dj;
      }
    }
    block_sum3<BT>(ch, dd, ddp, red);  // its barriers also end every read of xs
    const bool restart = stop_update(st, o, ch, dd, ddp, rs, have_check,
                                     sizeof(T) == 4 ? 5.9604644775390625e-8 : 1.1102230246251565e-16);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int j0 = (tid + BT * q) * VN;
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        if (j0 + e < n) xs[j0 + e] = restart ? static_cast<T>(1.0 / n) : xn[q][e];
        if (restart) dprev[q][e] = 0.0;
      }
    }
    __syncthreads();
    if (st.done) break;
    if (st.total_iter >= dense_cap) {
      // out of dense sweeps: the iterate and the stop state go to the
      // float64 continuation on the factored product
      for (int j = tid; j < n; j += BT) xbuf[m.vec_off + j] = xs[j];
      if (tid == 0) {
        SolveState out;
        out.s = st;
        out.sum_y = 0.0;
        out.pad = 0.0;
        states[pq] = out;
      }
      return;
    }

    // ---- a4: next sweep (a5: float64 check sweep when due) --------------
    have_check = st.check_next != 0;
    if (!have_check) {
#pragma unroll
      for (int q = 0; q < CPT; ++q)
#pragma unroll
        for (int e = 0; e < VN; ++e) acc[q][e] = cmp[q][e] = T(0);
      sweep_rows<T, BT, CPT, UE, false>(mat, ld, n, jc, xs, acc, cmp);
    } else {
#pragma unroll
      for (int q = 0; q < CPT; ++q)
#pragma unroll
        for (int e = 0; e < VN; ++e) accd[q][e] = dd0[q][e] = 0.0;
      sweep_rows<T, BT, CPT, UE, true>(mat, ld, n, jc, xs, accd, dd0);
    }
  }

  // ---- outputs --------------------------------------------------------------
  for (int j = tid; j < n; j += BT) pi_packed[m.pi_off + j] = xs[j];
  if (tid == 0) {
    infos[m.index] = make_info(st);
    states[pq].s.done = 1;  // nothing for the continuation
  }
  };

  if (!queue) {  // one workgroup per pixel
    solve(sel[blockIdx.x]);
    return;
  }
  // persistent workgroups: each takes the next pixel in launch order until
  // the queue is past the last one (every workgroup reaches that exit)
  for (;;) {
    __syncthreads();  // the previous pixel's reads of LDS and of next_pixel are done
    if (threadIdx.x == 0) next_pixel = atomicAdd(queue, 1);
    __syncthreads();
    const int idx = next_pixel;
    if (idx >= count) break;
    solve(sel[idx]);
  }
}

// ============================================================================
// Banded path for pixels too large for one block: a sweep is one launch over
// (pixel, row band, column block) items, each writing float64 partial sums of
// x P~ over its band; a combine launch (one block per pixel) adds the bands
// in order, normalises and applies the stop rule.  The first sweep builds the
// band's rows (shift fused) while it accumulates.  Launch boundaries order
// the steps, so no block ever waits for another.
// ============================================================================

// Whether banded sweep t (and its combine) runs.  The first sweep, which
// builds, always does; a later one only while the work items of the pixels
// still running after the previous sweep (counted by k_band_finish in
// live[t - 1]) number at least min_items, or always when min_items is 0.
// Every workgroup of the three launches reads the same count, so a sweep
// runs or is skipped as a whole, and once one is skipped every later one is
// (no count is taken in a skipped sweep).
__device__ inline bool band_sweep_runs(const int32_t* live, int t, int min_items) {
  return t == 0 || min_items == 0 ||
         __hip_atomic_load(live + t - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= min_items;
}

template <typename T, int BT>
__global__ __launch_bounds__(BT) void k_band_init(const PixelMeta* __restrict__ metas,
                                                  const int32_t* __restrict__ big,
                                                  const T* __restrict__ x0_packed,
                                                  T* __restrict__ xbuf, double* __restrict__ dprev,
                                                  SolveState* __restrict__ states, int start_flux,
                                                  int32_t* __restrict__ live, int nsweeps) {
  __shared__ double red[3 * BT / kWave];
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t < nsweeps; t += BT) live[t] = 0;
  const int q = big[blockIdx.x];
  const PixelMeta m = metas[q];
  const int n = m.n;
  double sum = 0.0, bad = 0.0;
  if (x0_packed) {
    for (int j = threadIdx.x; j < n; j += BT) {
      const double v = static_cast<double>(x0_packed[m.pi_off + j]);
      if (!(v >= 0.0) || !isfinite(v)) bad += 1.0;
      else sum += v;
    }
  }
  block_sum2<BT>(sum, bad, red);
  const bool warm = x0_packed && bad == 0.0 && sum > 0.0 && isfinite(sum);
  double fsum = 0.0, unused = 0.0;
  if (!x0_packed && start_flux) {
    for (int j = threadIdx.x; j < n; j += BT) fsum += start_flux_value(m, j);
    block_sum2<BT>(fsum, unused, red);
  }
  // as in start_vector: no usable flux at the centres falls back to uniform
  const bool flux = !x0_packed && start_flux && fsum > 0.0 && isfinite(fsum);
  for (int j = threadIdx.x; j < n; j += BT) {
    xbuf[m.vec_off + j] =
        warm ? static_cast<T>(static_cast<double>(x0_packed[m.pi_off + j]) / sum)
             : flux ? static_cast<T>(start_flux_value(m, j) / fsum) : static_cast<T>(1.0 / n);
    dprev[m.vec_off + j] = 0.0;
  }
  if (threadIdx.x == 0) {
    SolveState st;
    stop_init(st.s, warm ? 1 : 0, (x0_packed && !warm) ? DTM_INFO_WARM_REJECTED : 0);
    st.sum_y = 0.0;
    st.pad = 0.0;
    states[q] = st;
  }
}

template <typename T, int BT, int CPT>
__global__ __launch_bounds__(BT) void k_band_sweep(const PixelMeta* __restrict__ metas,
                                                   const BandItem* __restrict__ items,
                                                   const T* __restrict__ colf,
                                                   const double* __restrict__ scal,
                                                   const T* __restrict__ invs,
                                                   T* __restrict__ pool,
                                                   const T* __restrict__ xbuf,
                                                   const SolveState* __restrict__ states,
                                                   double* __restrict__ part, int band_rows,
                                                   const int32_t* __restrict__ live, int t, int min_items) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  // 16 column vectors in flight per thread (twice the one-block solver's):
  // once most pixels have converged, the last ones are swept by a handful of
  // items, and an item's rate is bounded by the bytes it keeps in flight.
  constexpr int UE = 16 / CPT;
  extern __shared__ __align__(16) unsigned char smem[];
  T* xs = reinterpret_cast<T*>(smem);
  if (!band_sweep_runs(live, t, min_items)) return;
  const bool first = t == 0;
  const BandItem it = items[blockIdx.x];
  const PixelMeta m = metas[it.meta];
  const StopState& st = states[it.meta].s;
  if (st.done) return;
  const bool check = st.check_next != 0;
  const int n = m.n;
  const int64_t ld = m.ld;
  const int i0 = it.band * band_rows;
  const int nr = min(band_rows, n - i0);
  const int tid = threadIdx.x;
  for (int r = tid; r < nr; r += BT) xs[r] = xbuf[m.vec_off + i0 + r];
  __syncthreads();
  const int cbase = it.colblock * (BT * VN * CPT);
  int jc[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int j0 = cbase + (tid + BT * q) * VN;
    jc[q] = j0 < n ? j0 : 0;
  }
  T* mat = pool + m.mat_off + static_cast<int64_t>(i0) * ld;
  T acc[CPT][VN], cmp[CPT][VN];
  double accd[CPT][VN], dd0[CPT][VN];
#pragma unroll
  for (int q = 0; q < CPT; ++q)
#pragma unroll
    for (int e = 0; e < VN; ++e) {
      acc[q][e] = cmp[q][e] = T(0);
      accd[q][e] = dd0[q][e] = 0.0;
    }
  if (first) {
    const T c = static_cast<T>(scal[it.meta]);
    T gr[CPT][VN];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int j0 = cbase + (tid + BT * q) * VN;
#pragma unroll
      for (int e = 0; e < VN; ++e) gr[q][e] = (j0 < n) ? colf[m.vec_off + j0 + e] : T(0);
    }
    for (int r = 0; r < nr; ++r) {
      const int i = i0 + r;
      int k = i + m.l;
      if (k >= n) k -= n;
      const T s = invs[m.vec_off + k];
      const T xi = xs[r];
      T* row = mat + static_cast<int64_t>(r) * ld;
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int j0 = cbase + (tid + BT * q) * VN;
        V v;
#pragma unroll
        for (int e = 0; e < VN; ++e) {
          v[e] = gr[q][e] * ((j0 + e) < k ? c : T(1)) * s;
          comp_add(acc[q][e], cmp[q][e], xi * v[e]);
        }
        if (j0 < n) __builtin_nontemporal_store(v, reinterpret_cast<V*>(row + j0));
      }
    }
  } else if (!check) {
    sweep_rows<T, BT, CPT, UE, false>(mat, ld, nr, jc, xs, acc, cmp);
  } else {
    sweep_rows<T, BT, CPT, UE, true>(mat, ld, nr, jc, xs, accd, dd0);
  }
  double* out = part + m.part_off + static_cast<int64_t>(it.band) * ld;
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int j0 = cbase + (tid + BT * q) * VN;
#pragma unroll
    for (int e = 0; e < VN; ++e)
      if (j0 + e < n)
        out[j0 + e] = check ? accd[q][e] : static_cast<double>(acc[q][e]) - static_cast<double>(cmp[q][e]);
  }
}

// Column j's partial sums of `bands` row bands (stride ld), added in band
// order.  Eight loads are issued ahead of their adds, so the dependent chain
// of additions does not wait on each load in turn; the order of the
// additions, and so the result, is that of the plain loop.
__device__ inline double band_sum(const double* __restrict__ p, int64_t ld, int bands) {
  double s = 0.0;
  int b = 0;
  for (; b + 8 <= bands; b += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[static_cast<int64_t>(b + u) * ld];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; b < bands; ++b) s += p[static_cast<int64_t>(b) * ld];
  return s;
}

// band_sum for the U columns j + BT u of one thread at once (8 U loads in
// flight).  Columns at or past n read column n - 1 instead; their sums are
// not used.
template <int U, int BT>
__device__ inline void band_sums(const double* __restrict__ p, int64_t ld, int bands, int j, int n,
                                 double (&y)[U]) {
  int jc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    jc[u] = min(j + BT * u, n - 1);
    y[u] = 0.0;
  }
  int b = 0;
  for (; b + 8 <= bands; b += 8) {
    double v[U][8];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < 8; ++k) v[u][k] = p[static_cast<int64_t>(b + k) * ld + jc[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < 8; ++k) y[u] += v[u][k];
  }
  for (; b < bands; ++b)
#pragma unroll
    for (int u = 0; u < U; ++u) y[u] += p[static_cast<int64_t>(b) * ld + jc[u]];
}

// The combine of a banded sweep in two launches, so that it is spread over
// the chip rather than one block per pixel (a pixel of 8192 bins has 8 x
// 8192 partial sums).  Stage 1, one block per column block of a banded
// pixel: y_j = the band partial sums of column j added in band order (eight
// loads in flight), stored in ybuf, and the block's sums of y and |y - x|.
template <typename T, int BT>
__global__ __launch_bounds__(BT) void k_band_colsum(const PixelMeta* __restrict__ metas,
                                                    const BandItem* __restrict__ citems,
                                                    const double* __restrict__ part,
                                                    const T* __restrict__ xbuf,
                                                    const SolveState* __restrict__ states,
                                                    double* __restrict__ ybuf, double* __restrict__ bsum,
                                                    int colw, const int32_t* __restrict__ live, int t,
                                                    int min_items) {
  __shared__ double red[3 * BT / kWave];
  if (!band_sweep_runs(live, t, min_items)) return;
  const BandItem it = citems[blockIdx.x];
  const PixelMeta m = metas[it.meta];
  if (states[it.meta].s.done) return;  // the same for every block of the pixel
  const double* pp = part + m.part_off;
  const T* x = xbuf + m.vec_off;
  double* y = ybuf + m.vec_off;
  const int c0 = it.colblock * colw, c1 = min(c0 + colw, m.n);
  constexpr int UC = 4;
  double sy = 0.0, rs = 0.0;
  for (int j0 = c0 + static_cast<int>(threadIdx.x); j0 < c1; j0 += UC * BT) {
    double yv[UC];
    band_sums<UC, BT>(pp, m.ld, m.bands, j0, c1, yv);
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int j = j0 + BT * u;
      if (j < c1) {
        y[j] = yv[u];
        sy += yv[u];
        rs += fabs(yv[u] - static_cast<double>(x[j]));
      }
    }
  }
  block_sum2<BT>(sy, rs, red);
  if (threadIdx.x == 0) {
    bsum[2 * blockIdx.x] = sy;
    bsum[2 * blockIdx.x + 1] = rs;
  }
}

// Stage 2, one block per banded pixel: sum y and the residual from the
// column blocks' sums (in column-block order), then the new iterate
// y / sum y, its change, and the stop rule.
template <typename T, int BT>
__global__ __launch_bounds__(BT) void k_band_finish(const PixelMeta* __restrict__ metas,
                                                    const int32_t* __restrict__ big,
                                                    const int32_t* __restrict__ cbase,
                                                    const double* __restrict__ ybuf,
                                                    const double* __restrict__ bsum, T* __restrict__ xbuf,
                                                    double* __restrict__ dprev, SolveState* __restrict__ states,
                                                    T* __restrict__ pi_packed, dtm_solve_info* __restrict__ infos,
                                                    KOpts o, int colw, int32_t* __restrict__ live, int t,
                                                    int min_items) {
  __shared__ double red[3 * BT / kWave];
  if (!band_sweep_runs(live, t, min_items)) return;
  const int q = big[blockIdx.x];
  const PixelMeta m = metas[q];
  StopState s = states[q].s;
  if (s.done) return;
  const bool was_check = s.check_next != 0;
  const int n = m.n;
  const int nb = (n + colw - 1) / colw;
  const double* bs = bsum + 2 * static_cast<int64_t>(cbase[m.big]);
  double sy = 0.0, rs = 0.0;
  for (int b = 0; b < nb; ++b) {
    sy += bs[2 * b];
    rs += bs[2 * b + 1];
  }
  const double inv = 1.0 / sy;
  const double* y = ybuf + m.vec_off;
  T* x = xbuf + m.vec_off;
  double* dp = dprev + m.vec_off;
  // columns j = tid, tid + BT, ... in that order, four loaded at a time
  constexpr int UC = 4;
  double ch = 0.0, dd = 0.0, ddp = 0.0;
  for (int j0 = threadIdx.x; j0 < n; j0 += UC * BT) {
    double yv[UC], xv[UC], pv[UC];
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int j = min(j0 + BT * u, n - 1);
      yv[u] = y[j];
      xv[u] = static_cast<double>(x[j]);
      pv[u] = dp[j];
    }
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int j = j0 + BT * u;
      if (j < n) {
        const T xn = static_cast<T>(yv[u] * inv);
        const double dj = static_cast<double>(xn) - xv[u];
        ch += fabs(dj);
        dd += dj * dj;
        ddp += dj * pv[u];
        dp[j] = dj;
        x[j] = xn;  // each thread owns its j: no other thread reads it in this launch
      }
    }
  }
  block_sum3<BT>(ch, dd, ddp, red);
  const bool restart = stop_update(s, o, ch, dd, ddp, rs, was_check,
                                   sizeof(T) == 4 ? 5.9604644775390625e-8 : 1.1102230246251565e-16);
  if (restart) {
    for (int j = threadIdx.x; j < n; j += BT) {
      x[j] = static_cast<T>(1.0 / n);
      dp[j] = 0.0;
    }
  }
  if (s.done) {
    for (int j = threadIdx.x; j < n; j += BT) pi_packed[m.pi_off + j] = x[j];
    if (threadIdx.x == 0) infos[m.index] = make_info(s);
  }
  if (threadIdx.x == 0) {
    SolveState out;
    out.s = s;
    out.sum_y = sy;
    out.pad = 0.0;
    states[q] = out;
    if (min_items > 0 && !s.done) atomicAdd(live + t, m.bands * nb);  // this pixel's items in sweep t + 1
  }
}

// ============================================================================
// Float64 refinement of the pixels a float32 solve could not certify (they
// stalled at the float32 round-off floor above the tolerance).  A
// slowly mixing chain (|lambda_2| near 1) amplifies the float32 round-off of
// the matrix and of the iterate by about 1 / (1 - |lambda_2|); when the
// float64 residual bound cannot reach the tolerance the pixel is re-solved
// here in float64, starting from its float32 result.  The matrix entries
// g_j w_kj / S_k are regenerated in every sweep from float64 tables held in
// LDS, so no float64 matrix is stored.  Thread t owns columns t + BT q.
// ============================================================================

template <int BT, int QMAX, typename TO>
__global__ __launch_bounds__(BT) void k_refine_f64(const PixelMeta* __restrict__ metas,
                                                   TO* __restrict__ pi_packed,
                                                   dtm_solve_info* __restrict__ infos, KOpts o,
                                                   int lds_ld) {
  const PixelMeta m = metas[blockIdx.x];
  const dtm_solve_info prev = infos[m.index];
  if (prev.status == DTM_OK || !(prev.flags & DTM_INFO_STALLED)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  double* g = reinterpret_cast<double*>(smem);  // tables, then u_i = x_i / S_{k(i)}
  double* invs = g + lds_ld;
  double* red = invs + lds_ld;
  const int n = m.n;
  const int tid = threadIdx.x;
  const double Lam = pixel_tables<double, BT>(m, g, nullptr, nullptr, red);
  const double c = exp(-Lam);
  __syncthreads();
  for (int k = tid / kWave; k < n; k += BT / kWave) {
    const double sk = wave_row_sum<double>(g, n, k, c);
    if ((tid % kWave) == 0) invs[k] = 1.0 / sk;
  }
  double gr[QMAX], xr[QMAX], dp[QMAX];
  double sum0 = 0.0, bad = 0.0;
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int j = tid + BT * q;
    gr[q] = (j < n) ? g[j] : 0.0;
    xr[q] = (j < n) ? static_cast<double>(pi_packed[m.pi_off + j]) : 0.0;
    dp[q] = 0.0;
    if (j < n) {
      if (!(xr[q] >= 0.0) || !isfinite(xr[q])) bad += 1.0;
      else sum0 += xr[q];
    }
  }
  block_sum2<BT>(sum0, bad, red);  // also orders the g reads before g is reused
  const bool start_ok = bad == 0.0 && sum0 > 0.0 && isfinite(sum0);
#pragma unroll
  for (int q = 0; q < QMAX; ++q) xr[q] = start_ok ? xr[q] / sum0 : 1.0 / n;
  StopState st;
  stop_init(st, 0, 0);
  double* u = g;
  for (;;) {
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int i = tid + BT * q;
      if (i < n) {
        int k = i + m.l;
        if (k >= n) k -= n;
        u[i] = xr[q] * invs[k];
      }
    }
    __syncthreads();
    double acc[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) acc[q] = 0.0;
    for (int i = 0; i < n; ++i) {
      int k = i + m.l;
      if (k >= n) k -= n;
      const double ui = u[i];
#pragma unroll
      for (int q = 0; q < QMAX; ++q) acc[q] += ui * ((tid + BT * q) < k ? c : 1.0);
    }
    double sy = 0.0, rs = 0.0;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      acc[q] *= gr[q];  // y_j
      if (tid + BT * q < n) {
        sy += acc[q];
        rs += fabs(acc[q] - xr[q]);
      }
    }
    block_sum2<BT>(sy, rs, red);
    double ch = 0.0, dd = 0.0, ddp = 0.0;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const double xn = acc[q] / sy;
      const double dj = (tid + BT * q < n) ? xn - xr[q] : 0.0;
      ch += fabs(dj);
      dd += dj * dj;
      ddp += dj * dp[q];
      dp[q] = dj;
      xr[q] = xn;
    }
    block_sum3<BT>(ch, dd, ddp, red);  // its barriers end the reads of u
    stop_update(st, o, ch, dd, ddp, rs, true, 1.1102230246251565e-16);
    if (st.done) break;
  }
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int j = tid + BT * q;
    if (j < n) pi_packed[m.pi_off + j] = static_cast<TO>(xr[q]);
  }
  if (tid == 0) {
    dtm_solve_info info = make_info(st);
    info.iterations += prev.iterations;
    info.dense_sweeps = prev.dense_sweeps;
    info.flags |= (prev.flags & ~(DTM_INFO_STALLED)) | DTM_INFO_REFINED;
    infos[m.index] = info;
  }
}

// ============================================================================
// Single-pixel power iteration on a caller's matrix (any row-stochastic P,
// any ld): a band kernel writes float64 partial sums of x P over row bands,
// a one-block combine kernel sums them in band order and applies the stop
// rule.  The host re-launches the pair and polls the state.
// ============================================================================

template <typename T, int BT>
__global__ __launch_bounds__(BT) void k_solver_init(const T* x0, T* x, double* dprev,
                                                    SolveState* state, int n) {
  __shared__ double red[3 * BT / kWave];
  double sum = 0.0, bad = 0.0;
  if (x0) {
    for (int j = threadIdx.x; j < n; j += BT) {
      const double v = static_cast<double>(x0[j]);
      if (!(v >= 0.0) || !isfinite(v)) bad += 1.0;
      else sum += v;
    }
  }
  block_sum2<BT>(sum, bad, red);
  const bool warm = x0 && bad == 0.0 && sum > 0.0 && isfinite(sum);
  for (int j = threadIdx.x; j < n; j += BT) {
    x[j] = warm ? static_cast<T>(static_cast<double>(x0[j]) / sum) : static_cast<T>(1.0 / n);
    dprev[j] = 0.0;
  }
  if (threadIdx.x == 0) {
    SolveState s;
    stop_init(s.s, warm ? 1 : 0, (x0 && !warm) ? DTM_INFO_WARM_REJECTED : 0);
    s.sum_y = 0.0;
    s.pad = 0.0;
    *state = s;
  }
}

// sum_{i0 <= i < i1} x_i P[i, j0 .. j0 + VN) in row order (float32
// compensated into acc/cmp, or float64 into accd on a check sweep), with
// sixteen rows' loads issued ahead of their adds: a small matrix is swept
// by few workgroups, and with one load in flight per thread each would wait
// on memory latency row after row.  The order of the additions, and so the
// result, is that of the plain row loop.
template <typename T, int VN>
__device__ inline void band_dot(const T* __restrict__ P, int64_t ld, int i0, int i1, int j0,
                                const T* __restrict__ x, bool check, T (&acc)[VN], T (&cmp)[VN],
                                double (&accd)[VN]) {
  using V = typename Vec<T>::type;
  constexpr int U = 16;
  int i = i0;
  for (; i + U <= i1; i += U) {
    V v[U];
    T xi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = *reinterpret_cast<const V*>(P + static_cast<int64_t>(i + u) * ld + j0);
      xi[u] = x[i + u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (check) {
#pragma unroll
        for (int e = 0; e < VN; ++e) accd[e] += static_cast<double>(xi[u]) * static_cast<double>(v[u][e]);
      } else {
#pragma unroll
        for (int e = 0; e < VN; ++e) comp_add(acc[e], cmp[e], xi[u] * v[u][e]);
      }
    }
  }
  for (; i < i1; ++i) {
    const V v = *reinterpret_cast<const V*>(P + static_cast<int64_t>(i) * ld + j0);
    const T xi = x[i];
    if (check) {
#pragma unroll
      for (int e = 0; e < VN; ++e) accd[e] += static_cast<double>(xi) * static_cast<double>(v[e]);
    } else {
#pragma unroll
      for (int e = 0; e < VN; ++e) comp_add(acc[e], cmp[e], xi * v[e]);
    }
  }
}

// Partial sums part[b][j] = sum_{i in band b} x_i P[i, j] for the column
// block blockIdx.x (BT * VN columns); float32 is compensated, the check
// sweep is float64.
template <typename T, int BT, int VN>
__global__ __launch_bounds__(BT) void k_sweep_band(const T* __restrict__ P, int n, int64_t ld,
                                                   const T* __restrict__ x,
                                                   const SolveState* __restrict__ state,
                                                   double* __restrict__ part, int64_t part_ld,
                                                   int band_rows) {
  if (state->s.done) return;
  const bool check = state->s.check_next != 0;
  const int band = blockIdx.y;
  const int i0 = band * band_rows;
  const int i1 = min(i0 + band_rows, n);
  const int j0 = (blockIdx.x * BT + threadIdx.x) * VN;
  if (j0 >= n) return;
  const int ne = min(VN, n - j0);
  T acc[VN], cmp[VN];
  double accd[VN];
#pragma unroll
  for (int e = 0; e < VN; ++e) {
    acc[e] = cmp[e] = T(0);
    accd[e] = 0.0;
  }
  if (VN > 1 && ne == VN) {
    band_dot<T, VN>(P, ld, i0, i1, j0, x, check, acc, cmp, accd);
  } else {
    for (int i = i0; i < i1; ++i) {
      const T xi = x[i];
      for (int e = 0; e < ne; ++e) {
        const T v = P[static_cast<int64_t>(i) * ld + j0 + e];
        if (check)
          accd[e] += static_cast<double>(xi) * static_cast<double>(v);
        else
          comp_add(acc[e], cmp[e], xi * v);
      }
    }
  }
  double* out = part + static_cast<int64_t>(band) * part_ld + j0;
  for (int e = 0; e < ne; ++e)
    out[e] = check ? accd[e] : static_cast<double>(acc[e]) - static_cast<double>(cmp[e]);
}

// Single-pixel combine, stage 1 (one block per 256 columns): y_j = the band
// partial sums of column j added in band order, and the block's sums of y
// and |y - x| (a fixed order), for stage 2.
template <typename T, int BT>
__global__ __launch_bounds__(BT) void k_combine_cols(const double* __restrict__ part, int64_t part_ld,
                                                     int bands, int n, const T* __restrict__ x,
                                                     const SolveState* __restrict__ state,
                                                     double* __restrict__ y, double* __restrict__ bsum) {
  __shared__ double red[3 * BT / kWave];
  if (state->s.done) return;  // the same for every block
  const int j = blockIdx.x * BT + threadIdx.x;
  double sy = 0.0, rs = 0.0;
  if (j < n) {
    const double yj = band_sum(part + j, part_ld, bands);
    y[j] = yj;
    sy = yj;
    rs = fabs(yj - static_cast<double>(x[j]));
  }
  block_sum2<BT>(sy, rs, red);
  if (threadIdx.x == 0) {
    bsum[2 * blockIdx.x] = sy;
    bsum[2 * blockIdx.x + 1] = rs;
  }
}

// Stage 2 (one block): sum y and the residual from the blocks' sums, then
// the new iterate y / sum y, its change, and the stop rule.
template <typename T, int BT>
__global__ __launch_bounds__(BT) void k_combine_finish(const double* __restrict__ y,
                                                       const double* __restrict__ bsum, int cblocks, int n,
                                                       T* __restrict__ x, double* __restrict__ dprev,
                                                       SolveState* __restrict__ state, T* __restrict__ pi,
                                                       KOpts o) {
  __shared__ double red[3 * BT / kWave];
  StopState s = state->s;
  if (s.done) return;
  const bool was_check = s.check_next != 0;
  double sy = 0.0, rs = 0.0;
  for (int i = 0; i < cblocks; ++i) {
    sy += bsum[2 * i];
    rs += bsum[2 * i + 1];
  }
  const double inv = 1.0 / sy;
  double ch = 0.0, dd = 0.0, ddp = 0.0;
  // columns j = tid, tid + BT, ... in that order, four loaded at a time
  constexpr int UC = 4;
  for (int j0 = threadIdx.x; j0 < n; j0 += UC * BT) {
    double yv[UC], xv[UC], pv[UC];
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int j = min(j0 + BT * u, n - 1);
      yv[u] = y[j];
      xv[u] = static_cast<double>(x[j]);
      pv[u] = dprev[j];
    }
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int j = j0 + BT * u;
      if (j < n) {
        const T xn = static_cast<T>(yv[u] * inv);
        const double dj = static_cast<double>(xn) - xv[u];
        ch += fabs(dj);
        dd += dj * dj;
        ddp += dj * pv[u];
        dprev[j] = dj;
        x[j] = xn;  // each thread owns its j: no other thread reads it in this launch
      }
    }
  }
  block_sum3<BT>(ch, dd, ddp, red);
  const bool restart = stop_update(s, o, ch, dd, ddp, rs, was_check,
                                   sizeof(T) == 4 ? 5.9604644775390625e-8 : 1.1102230246251565e-16);
  if (restart) {
    for (int j = threadIdx.x; j < n; j += BT) {
      x[j] = static_cast<T>(1.0 / n);
      dprev[j] = 0.0;
    }
  }
  if (s.done)
    for (int j = threadIdx.x; j < n; j += BT) pi[j] = x[j];
  if (threadIdx.x == 0) {
    SolveState out;
    out.s = s;
    out.sum_y = sy;
    out.pad = 0.0;
    *state = out;
  }
}

}  // namespace dtm

// ============================================================================
// Host side
// ============================================================================

using namespace dtm;

namespace {

constexpr int kBT = 256;
constexpr int kRowsPerWave = 4;

int hip_ok(hipError_t e) { return e == hipSuccess ? DTM_OK : DTM_EHIP; }
int last_launch() { return hip_ok(hipGetLastError()); }

PixelMeta single_meta(const dtm_scene& s, dtm_dtype dt) {
  PixelMeta m;
  m.t_r = s.period_ns;
  m.tau = s.pulse_center_ns;
  m.sigma = s.pulse_sigma_ns;
  m.S = s.signal_flux;
  m.B = s.background_flux;
  m.n = s.n_bins;
  shift_bins(s, &m.l);
  m.frac = 0.0;
  m.lam_mode = 0;
  m.pad2 = 0;
  m.ld = padded_ld(s.n_bins, dt);
  m.index = 0;
  m.t_d = s.dead_time_ns;
  m.e_s = std::exp(-s.signal_flux);
  m.e_b = std::exp(-s.background_flux);
  m.bands = 0;
  m.big = -1;
  m.part_off = 0;
  m.pi_off = 0;
  m.vec_off = 0;
  m.mat_off = 0;
  m.out_off = 0;
  return m;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

template <typename T>
int launch_tables(const PixelMeta* metas, const PixelMeta& one, int np, T* colf, T* invs, double* pk,
                  double* scal, T* lam, double* F, hipStream_t st) {
  hipLaunchKernelGGL((k_tables<T, kBT>), dim3(np), dim3(kBT), 0, st, metas, one, colf, invs, pk, scal,
                     lam, F);
  return last_launch();
}

template <typename T>
int launch_build(const PixelMeta* metas, const PixelMeta& one, int np, int max_n, const T* colf,
                 const double* scal, const T* invs, T* out, int64_t ld, int shifted, int packed,
                 hipStream_t st) {
  const int rows_per_block = (kBT / kWave) * kRowsPerWave;
  dim3 grid((max_n + rows_per_block - 1) / rows_per_block, np);
  hipLaunchKernelGGL((k_build<T, kBT, kRowsPerWave>), grid, dim3(kBT), 0, st, metas, one, colf,
                     scal, invs, out, ld, shifted, packed);
  return last_launch();
}

template <typename T>
int launch_shift(const PixelMeta* metas, const PixelMeta& one, int np, int max_n, const T* src,
                 T* dst, int64_t ld, hipStream_t st) {
  const int rows_per_block = (kBT / kWave) * kRowsPerWave;
  dim3 grid((max_n + rows_per_block - 1) / rows_per_block, np);
  hipLaunchKernelGGL((k_shift<T, kBT, kRowsPerWave>), grid, dim3(kBT), 0, st, metas, one, src, dst, ld);
  return last_launch();
}

// Single pixel: tables + row sums into the workspace.
template <typename T>
int single_prepare(const dtm_scene& s, dtm_dtype dt, void* ws, size_t ws_bytes, T* lam, double* F,
                   PixelMeta* m_out, SingleLayout* L_out, hipStream_t st) {
  const PixelMeta m = single_meta(s, dt);
  const SingleLayout L = single_layout(s.n_bins, dt);
  if (!ws) return DTM_EINVAL;
  if (ws_bytes < L.total) return DTM_ENOSPACE;
  char* w = static_cast<char*>(ws);
  T* colf = reinterpret_cast<T*>(w + L.off_colf);
  T* invs = reinterpret_cast<T*>(w + L.off_invs);
  double* scal = reinterpret_cast<double*>(w + L.off_scal);
  double* pk = reinterpret_cast<double*>(w + L.off_dprev);
  const int rc = launch_tables<T>(nullptr, m, 1, colf, invs, pk, scal, lam, F, st);
  *m_out = m;
  *L_out = L;
  return rc;
}

template <typename T>
int single_build(const dtm_scene* s, dtm_dtype dt, void* P, int64_t ld, void* ws, size_t ws_bytes,
                 int shifted, hipStream_t st) {
  PixelMeta m;
  SingleLayout L;
  int rc = single_prepare<T>(*s, dt, ws, ws_bytes, nullptr, nullptr, &m, &L, st);
  if (rc) return rc;
  char* w = static_cast<char*>(ws);
  return launch_build<T>(nullptr, m, 1, m.n, reinterpret_cast<T*>(w + L.off_colf),
                         reinterpret_cast<double*>(w + L.off_scal),
                         reinterpret_cast<T*>(w + L.off_invs), static_cast<T*>(P), ld, shifted, 0, st);
}

// Sweeps until the stop rule is predicted to end a pixel, from the state
// the host last read: the change shrinks by the estimated contraction per
// sweep, the rule fires once the change passes its test, and a check sweep
// follows.  Only schedules the next poll; the device decides convergence.
int predicted_sweeps(const StopState& s, const KOpts& o) {
  const bool bound = o.stop_rule != DTM_STOP_CHANGE;
  const double need = bound ? o.safety * o.tol : o.tol;
  const double have = bound ? s.c1 * s.gain * (o.final_check ? s.contr : 1.0) : s.c1;
  const int check = o.final_check ? 1 : 0;
  if (s.check_next) return 1;
  if (!(have > need)) return 1 + check;
  if (!(s.contr > 0.0) || s.contr >= 0.999) return 1 << 20;
  return static_cast<int>(std::min(std::ceil(std::log(need / have) / std::log(s.contr)), 1e6)) + check;
}

template <typename T>
int single_solve(const T* P, int32_t n, int64_t ld, const KOpts& ko, int check_every, const T* x0,
                 T* pi, void* ws, dtm_solve_info* info, hipStream_t st, dtm_dtype dt) {
  const SingleLayout L = single_layout(n, dt);
  char* w = static_cast<char*>(ws);
  T* x = reinterpret_cast<T*>(w + L.off_x);
  SolveState* state = reinterpret_cast<SolveState*>(w + L.off_state);
  double* dprev = reinterpret_cast<double*>(w + L.off_dprev);
  double* part = reinterpret_cast<double*>(w + L.off_part);
  double* y = reinterpret_cast<double*>(w + L.off_y);
  double* bsum = reinterpret_cast<double*>(w + L.off_bsum);
  constexpr int VN = Vec<T>::n;
  const bool vec = (ld % VN == 0) && (reinterpret_cast<uintptr_t>(P) % 16 == 0);
  hipLaunchKernelGGL((k_solver_init<T, kBT>), dim3(1), dim3(kBT), 0, st, x0, x, dprev, state, n);
  int rc = last_launch();
  if (rc) return rc;
  const int vn = vec ? VN : 1;
  const int cols_per_block = kBT * vn;
  dim3 grid((n + cols_per_block - 1) / cols_per_block, L.bands);
  SolveState hs;
  // Each three launches are one sweep; after `done` they return at once.
  // The stop rule ends every solve within 2 * max_iter sweeps (one restart).
  // The host polls after check_every sweeps, then after as many as the stop
  // rule's estimates predict are left (at least one, at most 4 check_every).
  const int max_sweeps = 2 * ko.max_iter + 2;
  int launched = 0, chunk = check_every;
  for (;;) {
    for (int r = 0; r < chunk && launched < max_sweeps; ++r, ++launched) {
      if (vec)
        hipLaunchKernelGGL((k_sweep_band<T, kBT, VN>), grid, dim3(kBT), 0, st, P, n, ld, x, state,
                           part, static_cast<int64_t>(L.ld), L.band_rows);
      else
        hipLaunchKernelGGL((k_sweep_band<T, kBT, 1>), grid, dim3(kBT), 0, st, P, n, ld, x, state,
                           part, static_cast<int64_t>(L.ld), L.band_rows);
      hipLaunchKernelGGL((k_combine_cols<T, kBT>), dim3(L.cblocks), dim3(kBT), 0, st, part,
                         static_cast<int64_t>(L.ld), L.bands, n, x, state, y, bsum);
      hipLaunchKernelGGL((k_combine_finish<T, kBT>), dim3(1), dim3(kBT), 0, st, y, bsum, L.cblocks, n, x, dprev,
                         state, pi, ko);
    }
    rc = last_launch();
    if (rc) return rc;
    if (hipMemcpyAsync(&hs, state, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess) return DTM_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return DTM_EHIP;
    if (hs.s.done || launched >= max_sweeps) break;
    chunk = std::max(1, std::min(predicted_sweeps(hs.s, ko), 4 * check_every));
  }
  if (!hs.s.done) {
    hs.s.status = DTM_ENOTCONV;
    if (hipMemcpyAsync(pi, x, sizeof(T) * n, hipMemcpyDeviceToDevice, st) != hipSuccess) return DTM_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return DTM_EHIP;
  }
  if (info) {
    info->iterations = hs.s.total_iter;
    info->status = hs.s.status;
    info->flags = hs.s.flags;
    info->dense_sweeps = hs.s.total_iter;
    info->change_l1 = hs.s.c1;
    info->residual_l1 = hs.s.resid;
    info->rho_hat = hs.s.rho;
  }
  return DTM_OK;
}

// One-block batched solve, kernel instance by (dtype, block, columns per
// thread); phase 0 launches the build, phase 1 the sweeps.
template <typename T, int BT, int CPT>
int launch_fused_cpt(const dtm_plan* plan, int phase, int unroll, const PixelMeta* metas, const int32_t* sel,
                     int count, const T* colf, const double* scal, T* pool, const T* x0, T* pi,
                     dtm_solve_info* infos, int lds_ld, hipStream_t st) {
  const size_t red = 3 * BT / kWave * sizeof(double);
  const size_t lds_build = 3 * sizeof(T) * static_cast<size_t>(lds_ld) + red;
  const size_t lds_sweeps = sizeof(T) * static_cast<size_t>(lds_ld) + red;
  auto build = k_solve_build<T, BT, CPT>;
  void (*sweeps)(const PixelMeta*, const T*, const T*, const double*, T*, dtm_solve_info*, const int32_t*,
                 KOpts, int, int, T*, SolveState*, int*, int) = nullptr;
  switch (unroll) {
    case 2: sweeps = k_solve_sweeps<T, BT, CPT, 2>; break;
    case 4: sweeps = k_solve_sweeps<T, BT, CPT, 4>; break;
    default: sweeps = k_solve_sweeps<T, BT, CPT, 8>; break;
  }
  if (lds_build > 64 * 1024 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(build), hipFuncAttributeMaxDynamicSharedMemorySize,
                          static_cast<int>(lds_build)) != hipSuccess)
    return DTM_EHIP;
  if (lds_sweeps > 64 * 1024 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(sweeps), hipFuncAttributeMaxDynamicSharedMemorySize,
                          static_cast<int>(lds_sweeps)) != hipSuccess)
    return DTM_EHIP;
  char* w = static_cast<char*>(plan->ws);
  const T* invs = reinterpret_cast<const T*>(w + plan->off_invs);
  // the first sweep's sums: the float64 slots the banded path uses for its
  // previous differences (disjoint pixels) and the tables kernel as scratch
  // (finished before this launch)
  double* y1 = reinterpret_cast<double*>(w + plan->off_dprev);
  // persistent sweep workgroups (tile fused_blocks > 0) take pixels from a
  // counter that the build launch resets
  const int persistent = plan->tiles.fused_blocks > 0 && plan->tiles.fused_blocks < count;
  int* queue = persistent ? reinterpret_cast<int*>(w + plan->off_queue) : nullptr;
  if (phase == 0)
    hipLaunchKernelGGL(build, dim3(count), dim3(BT), lds_build, st, metas, colf, invs, scal, pool, x0, y1, sel,
                       lds_ld, plan->kopts.start_flux, queue);
  else
    hipLaunchKernelGGL(sweeps, dim3(persistent ? plan->tiles.fused_blocks : count), dim3(BT), lds_sweeps, st,
                       metas, pool, x0, y1, pi, infos, sel, plan->kopts, lds_ld,
                       plan->tiles.dense_sweeps < plan->kopts.max_iter ? plan->tiles.dense_sweeps : INT32_MAX,
                       reinterpret_cast<T*>(w + plan->off_xbuf), reinterpret_cast<SolveState*>(w + plan->off_state),
                       queue, count);
  return last_launch();
}

template <typename T, int BT>
int launch_fused_bt(const dtm_plan* plan, int phase, int cpt, const PixelMeta* metas, const int32_t* sel,
                    int count, const T* colf, const double* scal, T* pool, const T* x0, T* pi,
                    dtm_solve_info* infos, int lds_ld, hipStream_t st) {
  const int u = plan->tiles.fused_unroll;
  switch (cpt) {
    case 1:
      return launch_fused_cpt<T, BT, 1>(plan, phase, u, metas, sel, count, colf, scal, pool, x0, pi, infos,
                                        lds_ld, st);
    case 2:
      return launch_fused_cpt<T, BT, 2>(plan, phase, u, metas, sel, count, colf, scal, pool, x0, pi, infos,
                                        lds_ld, st);
    case 4:
      return launch_fused_cpt<T, BT, 4>(plan, phase, u, metas, sel, count, colf, scal, pool, x0, pi, infos,
                                        lds_ld, st);
    default:
      return DTM_ENOTSUP;
  }
}

// Float64 refinement pass over the pixels of a float32 solve that failed
// their certificate (blocks of certified pixels return at once).
template <typename T>
int launch_refine(const dtm_plan* plan, const PixelMeta* metas, T* pi, dtm_solve_info* infos,
                  hipStream_t st) {
  constexpr int BT = 512, QMAX = 16;
  if (plan->max_n > BT * QMAX) return DTM_OK;  // wider pixels keep their STALLED status
  const size_t lds = 2 * sizeof(double) * static_cast<size_t>(plan->max_ld) + 3 * BT / kWave * sizeof(double);
  auto kern = k_refine_f64<BT, QMAX, T>;
  if (lds > 64 * 1024) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            static_cast<int>(lds)) != hipSuccess)
      return DTM_EHIP;
  }
  hipLaunchKernelGGL(kern, dim3(plan->n_pixels), dim3(BT), lds, st, metas, pi, infos, plan->kopts,
                     plan->max_ld);
  return last_launch();
}

// Banded path: k_band_init (launched by the caller before the one-block
// solver is forked off, so that it does not queue behind that solver's
// long-running blocks), then dense_sweeps x (sweep over all items, combine).
template <typename T>
int launch_band_init(const dtm_plan* plan, const PixelMeta* metas, const T* x0, hipStream_t st) {
  constexpr int BT = 256;
  char* w = static_cast<char*>(plan->ws);
  const int32_t* big = reinterpret_cast<const int32_t*>(w + plan->off_big);
  T* xbuf = reinterpret_cast<T*>(w + plan->off_xbuf);
  double* dprev = reinterpret_cast<double*>(w + plan->off_dprev);
  SolveState* states = reinterpret_cast<SolveState*>(w + plan->off_state);
  int32_t* live = reinterpret_cast<int32_t*>(w + plan->off_live);
  const int nbig = static_cast<int>(plan->big_sel.size());
  hipLaunchKernelGGL((k_band_init<T, BT>), dim3(nbig), dim3(BT), 0, st, metas, big, x0, xbuf, dprev,
                     states, plan->kopts.start_flux, live, plan->tiles.dense_sweeps);
  return last_launch();
}

// Sweeps [t0, t1) of the banded path (sweep 0 builds the matrices).
template <typename T>
int launch_banded(const dtm_plan* plan, int t0, int t1, const PixelMeta* metas, const T* colf,
                  const double* scal, const T* invs, T* pool, T* pi, dtm_solve_info* infos, hipStream_t st) {
  constexpr int BT = 256;
  char* w = static_cast<char*>(plan->ws);
  const int32_t* big = reinterpret_cast<const int32_t*>(w + plan->off_big);
  const BandItem* items = reinterpret_cast<const BandItem*>(w + plan->off_items);
  T* xbuf = reinterpret_cast<T*>(w + plan->off_xbuf);
  double* dprev = reinterpret_cast<double*>(w + plan->off_dprev);
  double* part = reinterpret_cast<double*>(w + plan->off_part);
  SolveState* states = reinterpret_cast<SolveState*>(w + plan->off_state);
  const int nbig = static_cast<int>(plan->big_sel.size());
  const int nitems = static_cast<int>(plan->items.size());
  const BandItem* citems = reinterpret_cast<const BandItem*>(w + plan->off_citems);
  const int32_t* cbase = reinterpret_cast<const int32_t*>(w + plan->off_cbase);
  double* bsum = reinterpret_cast<double*>(w + plan->off_bsum);
  double* ybuf = reinterpret_cast<double*>(w + plan->off_ybuf);
  const int ncitems = static_cast<int>(plan->citems.size());
  const int colw = plan->band_threads * Vec<T>::n * plan->band_cpt;
  const size_t lds = sizeof(T) * static_cast<size_t>(plan->tiles.band_rows);
  int32_t* live = reinterpret_cast<int32_t*>(w + plan->off_live);
  const int mi = plan->tiles.band_min_items;
  int rc = DTM_OK;
  void (*sweep)(const PixelMeta*, const BandItem*, const T*, const double*, const T*, T*, const T*,
                const SolveState*, double*, int, const int32_t*, int, int) = nullptr;
  switch (plan->band_cpt) {
    case 1: sweep = k_band_sweep<T, BT, 1>; break;
    case 2: sweep = k_band_sweep<T, BT, 2>; break;
    default: sweep = k_band_sweep<T, BT, 4>; break;
  }
  for (int t = t0; t < t1; ++t) {
    if (t == 0 && !plan->build_items.empty()) {
      // the building sweep in one-vector column blocks: its writes spread
      // over more workgroups; the same partial sums
      hipLaunchKernelGGL((k_band_sweep<T, BT, 1>), dim3(static_cast<int>(plan->build_items.size())), dim3(BT),
                         lds, st, metas, reinterpret_cast<const BandItem*>(w + plan->off_build_items), colf,
                         scal, invs, pool, xbuf, states, part, plan->tiles.band_rows, live, t, mi);
    } else {
      hipLaunchKernelGGL(sweep, dim3(nitems), dim3(BT), lds, st, metas, items, colf, scal, invs, pool,
                         xbuf, states, part, plan->tiles.band_rows, live, t, mi);
    }
    hipLaunchKernelGGL((k_band_colsum<T, BT>), dim3(ncitems), dim3(BT), 0, st, metas, citems, part, xbuf,
                       states, ybuf, bsum, colw, live, t, mi);
    hipLaunchKernelGGL((k_band_finish<T, BT>), dim3(nbig), dim3(BT), 0, st, metas, big, cbase, ybuf, bsum, xbuf,
                       dprev, states, pi, infos, plan->kopts, colw, live, t, mi);
    rc = last_launch();
    if (rc) return rc;
  }
  return DTM_OK;
}

template <typename T>
int batched_solve(const dtm_plan* plan, const void* x0, void* pi, dtm_solve_info* infos,
                  hipStream_t st) {
  char* w = static_cast<char*>(plan->ws);
  const PixelMeta* metas = reinterpret_cast<const PixelMeta*>(w + plan->off_meta);
  const int32_t* small = reinterpret_cast<const int32_t*>(w + plan->off_small);
  T* pool = reinterpret_cast<T*>(w + plan->off_pool);
  T* colf = reinterpret_cast<T*>(w + plan->off_colf);
  T* invs = reinterpret_cast<T*>(w + plan->off_invs);
  double* scal = reinterpret_cast<double*>(w + plan->off_scal);
  const T* x0t = static_cast<const T*>(x0);
  T* pit = static_cast<T*>(pi);
  constexpr int VN = Vec<T>::n;
  PixelMeta dummy;
  std::memset(&dummy, 0, sizeof(dummy));
  double* pk = reinterpret_cast<double*>(w + plan->off_dprev);
  int rc = launch_tables<T>(metas, dummy, plan->n_pixels, colf, invs, pk, scal, nullptr, nullptr, st);
  if (rc) return rc;
  const int nsmall = static_cast<int>(plan->small_sel.size());
  const int nbig = static_cast<int>(plan->big_sel.size());
  // With both kinds of pixels, the one-block solver runs on the plan's second
  // stream alongside the banded launches, which leave most of the GPU idle
  // while a sweep's last bands and the combines finish.
  const bool fork = nsmall > 0 && nbig > 0;
  if (nbig > 0) {
    rc = launch_band_init<T>(plan, metas, x0t, st);
    if (rc) return rc;
  }
  hipStream_t fst = st;
  if (fork) {
    fst = static_cast<hipStream_t>(plan->aux_stream);
    if (hipEventRecord(static_cast<hipEvent_t>(plan->ev_fork), st) != hipSuccess) return DTM_EHIP;
    if (hipStreamWaitEvent(fst, static_cast<hipEvent_t>(plan->ev_fork), 0) != hipSuccess) return DTM_EHIP;
  }
  // columns per thread covering the largest one-block pixel; at most 4
  // vectors of columns per thread (more would spill), so wide pixels take
  // 512 threads
  int bt = plan->tiles.fused_threads, cpt = 1;
  if (nsmall > 0) {
    cpt = (plan->max_ld_small + bt * VN - 1) / (bt * VN);
    if (cpt > 4 && bt == 256) {
      bt = 512;
      cpt = (plan->max_ld_small + bt * VN - 1) / (bt * VN);
    }
    cpt = cpt <= 1 ? 1 : cpt <= 2 ? 2 : 4;
    if (cpt * bt * VN < plan->max_ld_small) return DTM_ENOTSUP;
  }
  const int lds_ld = plan->max_ld_small;
  const auto one_block = [&](int phase) {
    return bt == 512 ? launch_fused_bt<T, 512>(plan, phase, cpt, metas, small, nsmall, colf, scal, pool, x0t, pit,
                                               infos, lds_ld, fst)
                     : launch_fused_bt<T, 256>(plan, phase, cpt, metas, small, nsmall, colf, scal, pool, x0t, pit,
                                               infos, lds_ld, fst);
  };
  // Every matrix is written before any is swept (HBM serves a stream of
  // writes and then a stream of reads better than the two mixed): the
  // one-block builds and the banded first sweep (which builds), then the
  // one-block sweeps and the remaining banded sweeps; with both kinds of
  // pixels each stream waits for the other's builds before it sweeps.
  if (nsmall > 0) {
    rc = one_block(0);
    if (rc) return rc;
  }
  if (nbig > 0) {
    rc = launch_banded<T>(plan, 0, std::min(1, plan->tiles.dense_sweeps), metas, colf, scal, invs, pool, pit, infos,
                          st);
    if (rc) return rc;
  }
  if (fork && !plan->tiles.independent_paths) {
    hipEvent_t small_built = static_cast<hipEvent_t>(plan->ev_join);
    hipEvent_t big_built = static_cast<hipEvent_t>(plan->ev_fork);
    if (hipEventRecord(small_built, fst) != hipSuccess || hipEventRecord(big_built, st) != hipSuccess ||
        hipStreamWaitEvent(fst, big_built, 0) != hipSuccess || hipStreamWaitEvent(st, small_built, 0) != hipSuccess)
      return DTM_EHIP;
  }
  if (nsmall > 0) {
    rc = one_block(1);
    if (rc) return rc;
    // one-block pixels still running after dense_sweeps go on in float64
    if (plan->tiles.dense_sweeps < plan->kopts.max_iter) {
      rc = launch_dense_tail(plan, 0, pit, infos, fst);
      if (rc) return rc;
    }
  }
  if (nbig > 0) {
    rc = launch_banded<T>(plan, 1, plan->tiles.dense_sweeps, metas, colf, scal, invs, pool, pit, infos, st);
    if (rc) return rc;
    // pixels still running after the launched sweeps go on in float64
    rc = launch_dense_tail(plan, 1, pit, infos, st);
    if (rc) return rc;
  }
  if (fork) {
    if (hipEventRecord(static_cast<hipEvent_t>(plan->ev_join), fst) != hipSuccess) return DTM_EHIP;
    if (hipStreamWaitEvent(st, static_cast<hipEvent_t>(plan->ev_join), 0) != hipSuccess) return DTM_EHIP;
  }
  if (sizeof(T) == 8) return DTM_OK;
  return launch_refine<T>(plan, metas, pit, infos, st);
}

template <typename T>
int batched_tables_rowsums(const dtm_plan* plan, hipStream_t st) {
  char* w = static_cast<char*>(plan->ws);
  const PixelMeta* metas = reinterpret_cast<const PixelMeta*>(w + plan->off_meta);
  T* colf = reinterpret_cast<T*>(w + plan->off_colf);
  T* invs = reinterpret_cast<T*>(w + plan->off_invs);
  double* scal = reinterpret_cast<double*>(w + plan->off_scal);
  double* pk = reinterpret_cast<double*>(w + plan->off_dprev);
  PixelMeta dummy;
  std::memset(&dummy, 0, sizeof(dummy));
  return launch_tables<T>(metas, dummy, plan->n_pixels, colf, invs, pk, scal, nullptr, nullptr, st);
}

template <typename T>
int batched_build(const dtm_plan* plan, void* out, int shifted, hipStream_t st) {
  int rc = batched_tables_rowsums<T>(plan, st);
  if (rc) return rc;
  char* w = static_cast<char*>(plan->ws);
  const PixelMeta* metas = reinterpret_cast<const PixelMeta*>(w + plan->off_meta);
  PixelMeta dummy;
  std::memset(&dummy, 0, sizeof(dummy));
  return launch_build<T>(metas, dummy, plan->n_pixels, plan->max_n,
                         reinterpret_cast<T*>(w + plan->off_colf),
                         reinterpret_cast<double*>(w + plan->off_scal),
                         reinterpret_cast<T*>(w + plan->off_invs), static_cast<T*>(out), 0, shifted,
                         1, st);
}

// Single-pixel power iteration on a caller's matrix with the solver's
// workspace at ws (argument checks first; nothing is launched on an error).
int stationary_pdf_in(const void* P_dev, int32_t n, int64_t ld, dtm_dtype dt, const dtm_solve_opts* opt,
                      const void* x0_dev, void* pi_dev, void* ws, size_t ws_bytes, dtm_solve_info* info_host,
                      dtm_stream_t stream) {
  if (!P_dev || !pi_dev || !ws) return DTM_EINVAL;
  if (dt != DTM_F32 && dt != DTM_F64) return DTM_EINVAL;
  if (n < 2 || n > DTM_MAX_BINS || ld < n) return DTM_EINVAL;
  KOpts ko;
  int32_t ce = 4;
  int rc = fill_opts(opt, &ko, &ce);
  if (rc) return rc;
  if (ko.model) return DTM_EINVAL;  // discretisation flags describe a plan's matrices, not a given one
  const SingleLayout L = single_layout(n, dt);
  if (ws_bytes < L.total) return DTM_ENOSPACE;
  const size_t es = dtype_size(dt);
  if (overlaps(pi_dev, es * n, ws, L.total)) return DTM_EALIAS;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dt == DTM_F32)
    return single_solve<float>(static_cast<const float*>(P_dev), n, ld, ko, ce, static_cast<const float*>(x0_dev),
                               static_cast<float*>(pi_dev), ws, info_host, st, dt);
  return single_solve<double>(static_cast<const double*>(P_dev), n, ld, ko, ce,
                              static_cast<const double*>(x0_dev), static_cast<double*>(pi_dev), ws, info_host, st,
                              dt);
}

// The single-pixel solver's workspace for dtm_stationary_pdf_noalloc, sized
// for DTM_NOALLOC_MAX_BINS bins in either dtype.  Every GPU holds its own
// copy; host code reaches it only through the address hipGetSymbolAddress
// returns on that device (the array's name is a host-side stand-in).
constexpr size_t kNoallocBytes =
    std::max(single_layout(DTM_NOALLOC_MAX_BINS, DTM_F64).total, single_layout(DTM_NOALLOC_MAX_BINS, DTM_F32).total);
static_assert(kNoallocBytes <= DTM_NOALLOC_SCRATCH_BYTES, "no-allocation scratch larger than documented");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) on its first use.
int noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return DTM_EHIP;
  if (dev >= kMaxDevices) return DTM_ENOTSUP;
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = p;
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev]) return DTM_EHIP;
  *out = g_scratch_ptr[dev];
  return DTM_OK;
}

}  // namespace

extern "C" {

int dtm_bin_tables(const dtm_scene* s, dtm_dtype dt, void* lambda_dev, double* F_dev,
                   void* workspace_dev, size_t workspace_bytes, dtm_stream_t stream) {
  if (!s) return DTM_EINVAL;
  const int v = validate_scene(*s, dt);
  if (v) return v;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const PixelMeta m = single_meta(*s, dt);
  const SingleLayout L = single_layout(s->n_bins, dt);
  if (!workspace_dev) return DTM_EINVAL;
  if (workspace_bytes < L.total) return DTM_ENOSPACE;
  char* w = static_cast<char*>(workspace_dev);
  double* scal = reinterpret_cast<double*>(w + L.off_scal);
  double* pk = reinterpret_cast<double*>(w + L.off_dprev);
  if (dt == DTM_F32)
    return launch_tables<float>(nullptr, m, 1, reinterpret_cast<float*>(w + L.off_colf),
                                reinterpret_cast<float*>(w + L.off_invs), pk, scal,
                                static_cast<float*>(lambda_dev), F_dev, st);
  return launch_tables<double>(nullptr, m, 1, reinterpret_cast<double*>(w + L.off_colf),
                               reinterpret_cast<double*>(w + L.off_invs), pk, scal,
                               static_cast<double*>(lambda_dev), F_dev, st);
}

static int check_matrix_args(const dtm_scene* s, dtm_dtype dt, const void* P, int64_t ld) {
  if (!s || !P) return DTM_EINVAL;
  const int v = validate_scene(*s, dt);
  if (v) return v;
  if (ld < s->n_bins) return DTM_EINVAL;
  return DTM_OK;
}

int dtm_build_base(const dtm_scene* s, dtm_dtype dt, void* P_base_dev, int64_t ld,
                   void* workspace_dev, size_t workspace_bytes, dtm_stream_t stream) {
  const int v = check_matrix_args(s, dt, P_base_dev, ld);
  if (v) return v;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dt == DTM_F32) return single_build<float>(s, dt, P_base_dev, ld, workspace_dev, workspace_bytes, 0, st);
  return single_build<double>(s, dt, P_base_dev, ld, workspace_dev, workspace_bytes, 0, st);
}

int dtm_build_transition(const dtm_scene* s, dtm_dtype dt, void* P_dev, int64_t ld,
                         void* workspace_dev, size_t workspace_bytes, dtm_stream_t stream) {
  const int v = check_matrix_args(s, dt, P_dev, ld);
  if (v) return v;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dt == DTM_F32) return single_build<float>(s, dt, P_dev, ld, workspace_dev, workspace_bytes, 1, st);
  return single_build<double>(s, dt, P_dev, ld, workspace_dev, workspace_bytes, 1, st);
}

int dtm_apply_deadtime_shift(const dtm_scene* s, dtm_dtype dt, const void* P_base_dev, void* P_dev,
                             int64_t ld, dtm_stream_t stream) {
  int v = check_matrix_args(s, dt, P_base_dev, ld);
  if (v) return v;
  if (!P_dev) return DTM_EINVAL;
  const size_t bytes = dtype_size(dt) * static_cast<size_t>(ld) * (s->n_bins - 1) +
                       dtype_size(dt) * s->n_bins;
  if (overlaps(P_base_dev, bytes, P_dev, bytes)) return DTM_EALIAS;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const PixelMeta m = single_meta(*s, dt);
  if (dt == DTM_F32)
    return launch_shift<float>(nullptr, m, 1, m.n, static_cast<const float*>(P_base_dev),
                               static_cast<float*>(P_dev), ld, st);
  return launch_shift<double>(nullptr, m, 1, m.n, static_cast<const double*>(P_base_dev),
                              static_cast<double*>(P_dev), ld, st);
}

int dtm_stationary_pdf(const void* P_dev, int32_t n, int64_t ld, dtm_dtype dt,
                       const dtm_solve_opts* opt, const void* x0_dev, void* pi_dev,
                       void* workspace_dev, size_t workspace_bytes, dtm_solve_info* info_host,
                       dtm_stream_t stream) {
  return stationary_pdf_in(P_dev, n, ld, dt, opt, x0_dev, pi_dev, workspace_dev, workspace_bytes, info_host,
                           stream);
}

int dtm_stationary_pdf_noalloc(const void* P_dev, int32_t n, int64_t ld, dtm_dtype dt,
                               const dtm_solve_opts* opt, const void* x0_dev, void* pi_dev,
                               dtm_solve_info* info_host, dtm_stream_t stream) {
  if (n > DTM_NOALLOC_MAX_BINS) return DTM_ENOSPACE;
  void* ws = nullptr;
  const int rc = noalloc_scratch(&ws);
  if (rc) return rc;
  return stationary_pdf_in(P_dev, n, ld, dt, opt, x0_dev, pi_dev, ws, kNoallocBytes, info_host, stream);
}

int dtm_plan_bind(dtm_plan* plan, void* workspace_dev, size_t workspace_bytes, dtm_stream_t stream) {
  if (!plan || !workspace_dev) return DTM_EINVAL;
  if (workspace_bytes < plan->total_bytes) return DTM_ENOSPACE;
  if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0) return DTM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(workspace_dev);
  if (hipMemcpyAsync(w + plan->off_meta, plan->meta.data(), sizeof(PixelMeta) * plan->meta.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return DTM_EHIP;
  if (!plan->small_sel.empty() &&
      hipMemcpyAsync(w + plan->off_small, plan->small_sel.data(),
                     sizeof(int32_t) * plan->small_sel.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return DTM_EHIP;
  if (!plan->big_sel.empty() &&
      hipMemcpyAsync(w + plan->off_big, plan->big_sel.data(), sizeof(int32_t) * plan->big_sel.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return DTM_EHIP;
  if (!plan->items.empty() &&
      hipMemcpyAsync(w + plan->off_items, plan->items.data(), sizeof(BandItem) * plan->items.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return DTM_EHIP;
  if (!plan->build_items.empty() &&
      hipMemcpyAsync(w + plan->off_build_items, plan->build_items.data(),
                     sizeof(BandItem) * plan->build_items.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return DTM_EHIP;
  if (!plan->citems.empty() &&
      (hipMemcpyAsync(w + plan->off_citems, plan->citems.data(), sizeof(BandItem) * plan->citems.size(),
                      hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(w + plan->off_cbase, plan->cbase.data(), sizeof(int32_t) * plan->cbase.size(),
                      hipMemcpyHostToDevice, st) != hipSuccess))
    return DTM_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return DTM_EHIP;
  if (!plan->aux_stream) {
    hipStream_t aux;
    hipEvent_t a, b;
    if (hipStreamCreateWithFlags(&aux, hipStreamNonBlocking) != hipSuccess) return DTM_EHIP;
    if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(aux);
      return DTM_EHIP;
    }
    if (hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
      (void)hipEventDestroy(a);
      (void)hipStreamDestroy(aux);
      return DTM_EHIP;
    }
    plan->aux_stream = aux;
    plan->ev_fork = a;
    plan->ev_join = b;
  }
  plan->ws = workspace_dev;
  plan->ws_bytes = workspace_bytes;
  return DTM_OK;
}

void dtm_plan_destroy(dtm_plan* plan) {
  if (!plan) return;
  if (plan->aux_stream) {
    (void)hipStreamSynchronize(static_cast<hipStream_t>(plan->aux_stream));
    (void)hipStreamDestroy(static_cast<hipStream_t>(plan->aux_stream));
    (void)hipEventDestroy(static_cast<hipEvent_t>(plan->ev_fork));
    (void)hipEventDestroy(static_cast<hipEvent_t>(plan->ev_join));
  }
  delete plan;
}

int dtm_solve_batched(const dtm_plan* plan, const void* x0_packed_dev, void* pi_packed_dev,
                      dtm_solve_info* infos_dev, dtm_stream_t stream) {
  if (!plan || !plan->ws || !pi_packed_dev || !infos_dev) return DTM_EINVAL;
  if (plan->kopts.pad) return DTM_ENOTSUP;  // created with DTM_FLAG_NO_DENSE
  const size_t es = dtype_size(plan->dt);
  if (overlaps(pi_packed_dev, es * plan->pi_elems, plan->ws, plan->total_bytes)) return DTM_EALIAS;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (plan->dt == DTM_F32) return batched_solve<float>(plan, x0_packed_dev, pi_packed_dev, infos_dev, st);
  return batched_solve<double>(plan, x0_packed_dev, pi_packed_dev, infos_dev, st);
}

struct dtm_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

int dtm_graph_create(const dtm_plan* plan, const void* x0_packed_dev, void* pi_packed_dev,
                     dtm_solve_info* infos_dev, dtm_stream_t stream, dtm_graph** graph_out) {
  if (!graph_out) return DTM_EINVAL;
  *graph_out = nullptr;
  if (!plan || !plan->ws || !pi_packed_dev || !infos_dev) return DTM_EINVAL;
  if (plan->kopts.pad) return DTM_ENOTSUP;
  const size_t es = dtype_size(plan->dt);
  if (overlaps(pi_packed_dev, es * plan->pi_elems, plan->ws, plan->total_bytes)) return DTM_EALIAS;
  hipStream_t user = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(user) != hipSuccess) return DTM_EHIP;
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return DTM_EHIP;
  int rc = DTM_OK;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return DTM_EHIP;
  }
  rc = plan->dt == DTM_F32 ? batched_solve<float>(plan, x0_packed_dev, pi_packed_dev, infos_dev, cs)
                           : batched_solve<double>(plan, x0_packed_dev, pi_packed_dev, infos_dev, cs);
  const hipError_t ec = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (rc != DTM_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return rc != DTM_OK ? rc : DTM_EHIP;
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return DTM_EHIP;
  }
  dtm_graph* out = new (std::nothrow) dtm_graph{g, ex};
  if (!out) {
    (void)hipGraphExecDestroy(ex);
    (void)hipGraphDestroy(g);
    return DTM_EINVAL;
  }
  *graph_out = out;
  return DTM_OK;
}

int dtm_graph_launch(dtm_graph* graph, dtm_stream_t stream) {
  if (!graph) return DTM_EINVAL;
  return hip_ok(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
}

void dtm_graph_destroy(dtm_graph* graph) {
  if (!graph) return;
  (void)hipGraphExecDestroy(graph->exec);
  (void)hipGraphDestroy(graph->graph);
  delete graph;
}

int dtm_build_base_batched(const dtm_plan* plan, void* P_packed_dev, dtm_stream_t stream) {
  if (!plan || !plan->ws || !P_packed_dev) return DTM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (plan->dt == DTM_F32) return batched_build<float>(plan, P_packed_dev, 0, st);
  return batched_build<double>(plan, P_packed_dev, 0, st);
}

int dtm_build_transition_batched(const dtm_plan* plan, void* P_packed_dev, dtm_stream_t stream) {
  if (!plan || !plan->ws || !P_packed_dev) return DTM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (plan->dt == DTM_F32) return batched_build<float>(plan, P_packed_dev, 1, st);
  return batched_build<double>(plan, P_packed_dev, 1, st);
}

int dtm_apply_deadtime_shift_batched(const dtm_plan* plan, const void* P_base_packed_dev,
                                     void* P_packed_dev, dtm_stream_t stream) {
  if (!plan || !plan->ws || !P_base_packed_dev || !P_packed_dev) return DTM_EINVAL;
  const size_t bytes = dtype_size(plan->dt) * static_cast<size_t>(plan->mat_elems);
  if (overlaps(P_base_packed_dev, bytes, P_packed_dev, bytes)) return DTM_EALIAS;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(plan->ws);
  const PixelMeta* metas = reinterpret_cast<const PixelMeta*>(w + plan->off_meta);
  PixelMeta dummy;
  std::memset(&dummy, 0, sizeof(dummy));
  if (plan->dt == DTM_F32)
    return launch_shift<float>(metas, dummy, plan->n_pixels, plan->max_n,
                               static_cast<const float*>(P_base_packed_dev),
                               static_cast<float*>(P_packed_dev), 0, st);
  return launch_shift<double>(metas, dummy, plan->n_pixels, plan->max_n,
                              static_cast<const double*>(P_base_packed_dev),
                              static_cast<double*>(P_packed_dev), 0, st);
}

}  // extern "C"
