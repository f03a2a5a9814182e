// Monte Carlo simulation of the asynchronous SPAD with dead time (Section 2.1):
// Poisson photon arrivals of rate lambda(t) in every laser period, a
// non-paralyzable dead time after each registration, free-running rearm, and
// a histogram of X_k = T_k mod t_r.  It checks the Markov model against the
// physics it approximates (Section 3.5 compares with Monte Carlo the same way).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011), one
// stream per period: key = seed, counter = (draw block, period, run, pixel);
// a block gives four words w, read as u = (w + 1/2) / 2^32.  Block 0: the
// pulse and background counts (words 0, 1), Poisson draws by inversion of
// one uniform against cumulative probabilities built from exp(-S), exp(-B)
// (host libm) by the recurrence p_k = p_{k-1} mean / k.  Then one block per
// four pulse photons, two Box-Muller pairs tau + sigma sqrt(-2 ln u1)
// (cos, sin)(2 pi u2) as far as the count goes, kept inside [0, t_r); then
// one block per four background photons t_r u.  The detector state is the rearm time a relative
// to the period start (0 = armed): photons are visited in time order, one at
// t >= a is registered and sets a = t + t_d; the period ends with
// a = max(a - t_r, 0).
//
// A run is sequential only through a, so a group of L lanes simulates one
// run: each lane draws one period of a chunk of L periods (its own
// stream), then the group hands a from lane to lane through the chunk.  L = 1
// (a lane per run) has the highest throughput when runs fill the chip; L = 64
// (a wave per run) the lowest latency when there are few runs (a run's time
// is then set by its hand-over chain, not by its drawing).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "dtm_internal.h"

// Every product and sum below is rounded on its own (no fused multiply-add),
// so that the pulse times, period bases and dead-time comparisons are the
// ones any IEEE double implementation of the same steps computes.
#pragma clang fp contract(off)

namespace dtm {
namespace mc {

constexpr int BT = 64;        // one wave per block
constexpr int kCoopMin = 16;  // lanes per run from which the hand-over search is shared

__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// The four uniforms (w + 1/2) / 2^32 of draw block `block` of a period's
// stream: Philox4x32-10 of the counter (block, period, run, pixel).
struct Draws {
  uint32_t k0, k1, cycle, run, pixel;

  __device__ inline void block(uint32_t b, double u[4]) const {
    uint32_t w[4] = {b, cycle, run, pixel};
    philox4x32_10(w, k0, k1);
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = (static_cast<double>(w[q]) + 0.5) * (1.0 / 4294967296.0);
  }
};

constexpr int KMAX = 128;  // Poisson table length (counts above 127 read as 127)

// C_0 = p_0, p_k = p_{k-1} mean / k, C_k = C_{k-1} + p_k: the cumulative
// Poisson probabilities, summed in this order (one thread).
__device__ inline void poisson_cdf(double mean, double p0, double* cdf) {
  double p = p0, c = p0;
  cdf[0] = p0;
  for (int k = 1; k < KMAX; ++k) {
    p = p * mean / static_cast<double>(k);
    c = c + p;
    cdf[k] = c;
  }
}

// Poisson draw by inversion of one uniform: the first k with u <= C_k.
__device__ inline int poisson(double u, const double* cdf) {
  int k = 0;
  while (k < KMAX - 1 && u > cdf[k]) ++k;
  return k;
}

__global__ __launch_bounds__(BT) void k_zero(uint32_t* __restrict__ p, size_t n) {
  const size_t i = static_cast<size_t>(blockIdx.x) * BT + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Exclusive prefix sum over the wave.
__device__ inline int wave_exclusive_sum(int v, int lane) {
  int s = v;
#pragma unroll
  for (int d = 1; d < BT; d <<= 1) {
    const int u = __shfl_up(s, d, BT);
    if (lane >= d) s += u;
  }
  return s - v;
}

// Grid (pixel, run block); block = one wave = 64 / L runs of one pixel.
// LDS: a pool of `cap` photon times shared by the wave's 64 periods of a
// chunk (each lane owns a contiguous segment, placed by a prefix sum of its
// Poisson counts, sorted), for each photon the last registration of the
// chain that starts with it (uint16, same offsets), then the pixel's
// histogram (n uint32), added atomically to HBM at the end.
__global__ __launch_bounds__(BT) void k_mc(const PixelMeta* __restrict__ metas, int runs, int64_t cycles,
                                           int64_t burn, uint64_t seed, int L, int cap,
                                           uint32_t* __restrict__ hist, uint32_t* __restrict__ overflow) {
  extern __shared__ double lds_d[];
  __shared__ double cdf_s[KMAX], cdf_b[KMAX];
  double* pool = lds_d;
  uint16_t* jend = reinterpret_cast<uint16_t*>(lds_d + cap);
  uint32_t* h = reinterpret_cast<uint32_t*>(lds_d + cap) + (cap + 1) / 2;
  const PixelMeta m = metas[blockIdx.x];
  const int n = m.n;
  const int lane = threadIdx.x;
  for (int j = lane; j < n; j += BT) h[j] = 0u;
  if (lane == 0) poisson_cdf(m.S, m.e_s, cdf_s);
  if (lane == 1) poisson_cdf(m.B, m.e_b, cdf_b);
  __syncthreads();
  const int k_in = lane % L, base_lane = lane - k_in;
  const int run = blockIdx.y * (BT / L) + lane / L;
  const bool run_ok = run < runs;
  const double delta = m.t_r / n;
  const double two_pi = 2.0 * 3.141592653589793;
  bool over = false;
  double a = 0.0;  // rearm time of this lane's run, relative to the chunk's next period
  for (int64_t c0 = 0; c0 < cycles; c0 += L) {
    const int64_t c = c0 + k_in;
    const bool mine = run_ok && c < cycles;
    Draws st;
    st.k0 = static_cast<uint32_t>(seed);
    st.k1 = static_cast<uint32_t>(seed >> 32);
    st.cycle = static_cast<uint32_t>(c);
    st.run = static_cast<uint32_t>(run);
    st.pixel = static_cast<uint32_t>(m.index);
    int ns = 0, nb = 0;
    if (mine) {
      double u[4];
      st.block(0u, u);  // block 0: the two counts
      ns = poisson(u[0], cdf_s);
      nb = poisson(u[1], cdf_b);
    }
    const int off = wave_exclusive_sum(ns + nb, lane);
    const int room = min(ns + nb, max(cap - off, 0));
    double* seg = pool + off;
    int cnt = 0;
    if (mine) {
      // one block per four pulse photons (two Box-Muller pairs, whose
      // transcendental chains overlap), then one per four background photons
      uint32_t blk = 1u;
      for (int i = 0; i < ns; i += 4) {
        double u[4];
        st.block(blk++, u);
        const double ra = sqrt(-2.0 * log(u[0])), rb = sqrt(-2.0 * log(u[2]));
        double sna, csa, snb, csb;
        sincos(two_pi * u[1], &sna, &csa);
        sincos(two_pi * u[3], &snb, &csb);
        const double t[4] = {m.tau + m.sigma * (ra * csa), m.tau + m.sigma * (ra * sna),
                             m.tau + m.sigma * (rb * csb), m.tau + m.sigma * (rb * snb)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (i + q < ns && t[q] >= 0.0 && t[q] < m.t_r) {
            if (cnt < room) seg[cnt++] = t[q];
            else over = true;
          }
        }
      }
      for (int i = 0; i < nb; i += 4) {
        double u[4];
        st.block(blk++, u);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (i + q < nb) {
            if (cnt < room) seg[cnt++] = m.t_r * u[q];
            else over = true;
          }
        }
      }
      for (int x = 1; x < cnt; ++x) {  // insertion sort of this lane's segment
        const double v = seg[x];
        int y = x - 1;
        while (y >= 0 && seg[y] > v) {
          seg[y + 1] = seg[y];
          --y;
        }
        seg[y + 1] = v;
      }
      if (L >= kCoopMin) {
        // A registration at photon i is followed by one at the first photon
        // q > i with t_q >= t_i + t_d; q only moves left as i does.  jend[i]:
        // the last registration of the period once photon i is registered.
        int q = cnt;
        for (int i = cnt - 1; i >= 0; --i) {
          const double thr = seg[i] + m.t_d;
          while (q - 1 > i && seg[q - 1] >= thr) --q;
          jend[off + i] = static_cast<uint16_t>(q == cnt ? i : jend[off + q]);
        }
      }
    }
    double a_in = 0.0;
    if (L < kCoopMin) {
      // Small groups: the lane holding period c0 + k walks its own sorted
      // segment (entering at or before its first photon, the exit does not
      // depend on a and was found beforehand) and passes a on.
      double A0 = 0.0;
      if (mine && cnt > 0) {
        double aa = 0.0;
        for (int x = 0; x < cnt; ++x) {
          const double t = seg[x];
          if (t >= aa) aa = t + m.t_d;
        }
        A0 = fmax(aa - m.t_r, 0.0);
      }
      for (int k = 0; k < L; ++k) {
        if (mine && k_in == k) {
          a_in = a;
          if (cnt > 0 && a <= seg[0]) {
            a = A0;
          } else {
            for (int x = 0; x < cnt; ++x) {
              const double t = seg[x];
              if (t >= a) a = t + m.t_d;
            }
            a = fmax(a - m.t_r, 0.0);
          }
        }
        if (L > 1) a = __shfl(a, base_lane + k, BT);
      }
    } else {
      // Large groups: for period c0 + k the group's lanes look in parallel for
      // the first photon at or after a (the segment is sorted); the period's
      // exit rearm time follows from that photon's jend.
      const int cnt_or_none = mine ? cnt : -1;
      const uint64_t gmask = L == BT ? ~0ull : ((1ull << L) - 1ull);
      for (int k = 0; k < L; ++k) {
        const int src = base_lane + k;
        const int off_k = __shfl(off, src, BT);
        const int cnt_k = __shfl(cnt_or_none, src, BT);
        if (k_in == k) a_in = a;
        int first = cnt_k;
        bool searching = cnt_k > 0;
        for (int r0 = 0; __any(searching); r0 += L) {
          const int idx = r0 + k_in;
          const bool hit = searching && idx < cnt_k && pool[off_k + idx] >= a;
          const uint64_t g = (static_cast<uint64_t>(__ballot(hit)) >> base_lane) & gmask;
          if (searching) {
            if (g) {
              first = r0 + __ffsll(static_cast<unsigned long long>(g)) - 1;
              searching = false;
            } else if (r0 + L >= cnt_k) {
              searching = false;
            }
          }
        }
        if (cnt_k >= 0) {
          const double exit_from = first < cnt_k ? pool[off_k + jend[off_k + first]] + m.t_d : a;
          a = fmax(exit_from - m.t_r, 0.0);
        }
      }
    }
    // Registrations of every period of the chunk, in parallel.
    if (mine && c >= burn) {
      double aa = a_in;
      for (int x = 0; x < cnt; ++x) {
        const double t = seg[x];
        if (t >= aa) {
          aa = t + m.t_d;
          int j = static_cast<int>(ceil(t / delta)) - 1;
          if (j < 0) j += n;
          if (j >= n) j -= n;
          atomicAdd(&h[j], 1u);
        }
      }
    }
  }
  if (over) atomicOr(&overflow[m.index], 1u);
  __syncthreads();
  for (int j = lane; j < n; j += BT)
    if (h[j]) atomicAdd(&hist[m.pi_off + j], h[j]);
}

}  // namespace mc
}  // namespace dtm

using namespace dtm;

extern "C" int dtm_mc_histograms(const dtm_plan* plan, int32_t runs_per_pixel, int64_t cycles,
                                 int64_t burn_cycles, uint64_t seed, int32_t lanes_per_run,
                                 uint32_t* hist_packed_dev, uint32_t* overflow_dev, dtm_stream_t stream) {
  if (!plan || !plan->ws || !hist_packed_dev || !overflow_dev) return DTM_EINVAL;
  if (runs_per_pixel < 1 || runs_per_pixel > 65535 || cycles < 1 || cycles > 0xFFFFFFFFll ||
      burn_cycles < 0 || burn_cycles >= cycles)
    return DTM_EINVAL;
  if (static_cast<double>(runs_per_pixel) * static_cast<double>(cycles - burn_cycles) >= 67108864.0)
    return DTM_EINVAL;
  if (lanes_per_run < 0 || lanes_per_run > mc::BT || (lanes_per_run & (lanes_per_run - 1)))
    return DTM_EINVAL;
  if (plan->max_n > 16384) return DTM_ENOTSUP;
  for (const PixelMeta& m : plan->meta)
    if (m.S + m.B > 24.0) return DTM_ENOTSUP;
  int L = lanes_per_run;
  if (L == 0) {
    // At least 8 lanes per run, more until the runs give about one and a
    // half waves to each SIMD of the 256 CUs (measured: the longer hand-over
    // chain of a larger group costs less than an idle SIMD).
    const double chains = static_cast<double>(plan->n_pixels) * runs_per_pixel;
    L = 8;
    while (L < mc::BT && chains * L < 256.0 * 4 * 64 * 1.5) L *= 2;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const char* w = static_cast<const char*>(plan->ws);
  const PixelMeta* metas = reinterpret_cast<const PixelMeta*>(w + plan->off_meta);
  // Photon pool of a wave: the 64 periods of a chunk draw Poisson(S' + B)
  // photons in all, S' + B <= S + B; the pool holds that mean plus ten
  // standard deviations (a wave that draws more drops the excess and flags
  // the pixel).
  double lam = 0.0;
  for (const PixelMeta& m : plan->meta) lam = std::max(lam, m.S + m.B);
  const double mean = mc::BT * lam;
  const int cap = static_cast<int>(std::ceil(mean + 10.0 * std::sqrt(mean) + 64.0));
  const size_t lds = sizeof(double) * static_cast<size_t>(cap) + sizeof(uint32_t) * static_cast<size_t>((cap + 1) / 2) +
                    sizeof(uint32_t) * static_cast<size_t>(plan->max_n);
  if (lds > 160 * 1024) return DTM_ENOTSUP;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(mc::k_mc), hipFuncAttributeMaxDynamicSharedMemorySize,
                          static_cast<int>(lds)) != hipSuccess)
    return DTM_EHIP;
  const size_t total = plan->pi_elems;
  hipLaunchKernelGGL(mc::k_zero, dim3(static_cast<unsigned>((total + mc::BT - 1) / mc::BT)), dim3(mc::BT), 0, st,
                     hist_packed_dev, total);
  const int per_block = mc::BT / L;
  const unsigned run_blocks = static_cast<unsigned>((runs_per_pixel + per_block - 1) / per_block);
  hipLaunchKernelGGL(mc::k_mc, dim3(plan->n_pixels, run_blocks), dim3(mc::BT), lds, st, metas, runs_per_pixel,
                     cycles, burn_cycles, seed, L, cap, hist_packed_dev, overflow_dev);
  return hipGetLastError() == hipSuccess ? DTM_OK : DTM_EHIP;
}
