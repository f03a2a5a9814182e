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
// chain of periods: each lane draws one period of a chunk of L periods (its
// own stream), then the group hands a from lane to lane through the chunk.
//
// Few runs do not fill the chip, so a run may also be cut into K segments of
// consecutive periods, all simulated at once (k_mc), each from the armed
// state a = 0 instead of the unknown rearm time its predecessor leaves.
// Two trajectories of the detector that see the same photons agree from the
// first photon both register on (a registration sets a from the photon
// alone), and agree for good once their rearm times are equal at the start
// of a period.  So the counts are repaired exactly: k_mc_repair walks each
// segment again from the predecessor's speculative end (its true end when the
// predecessor itself coupled) beside the armed start, adding the first
// trajectory's registrations and removing the second's until the two
// coupled; the same pass then runs along each run in segment order and
// repeats the walk for every segment whose predecessor ended elsewhere
// (a predecessor that never coupled).  The histogram is then the one a single
// sequential walk of the run gives, count for count.
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

constexpr int BT = 64;        // wavefront size (one wavefront per block in the repair passes)
constexpr int WPB = 2;        // wavefronts per block of k_mc (they share the pixel's histogram)
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

__device__ inline Draws period_stream(uint64_t seed, int64_t c, int run, const PixelMeta& m) {
  Draws st;
  st.k0 = static_cast<uint32_t>(seed);
  st.k1 = static_cast<uint32_t>(seed >> 32);
  st.cycle = static_cast<uint32_t>(c);
  st.run = static_cast<uint32_t>(run);
  st.pixel = static_cast<uint32_t>(m.index);
  return st;
}

// Block 0 of a period: the pulse and background photon counts.
__device__ inline void period_counts(const Draws& st, const double* cdf_s, const double* cdf_b, int& ns, int& nb) {
  double u[4];
  st.block(0u, u);
  ns = poisson(u[0], cdf_s);
  nb = poisson(u[1], cdf_b);
}

// The period's photons inside [0, t_r) into seg (at most room of them, the
// rest dropped and *over set), sorted by time; returns how many were kept.
// One block per four pulse photons (two Box-Muller pairs, whose
// transcendental chains overlap), then one per four background photons.
__device__ inline int period_photons(const PixelMeta& m, const Draws& st, int ns, int nb, double* seg, int room,
                                     bool* over) {
  const double two_pi = 2.0 * 3.141592653589793;
  int cnt = 0;
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
        else *over = true;
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
        else *over = true;
      }
    }
  }
  for (int x = 1; x < cnt; ++x) {  // insertion sort
    const double v = seg[x];
    int y = x - 1;
    while (y >= 0 && seg[y] > v) {
      seg[y + 1] = seg[y];
      --y;
    }
    seg[y + 1] = v;
  }
  return cnt;
}

// Bin of a registration at time t in [0, t_r): ceil(t / Delta) - 1, mod n.
__device__ inline int bin_of(double t, double delta, int n) {
  int j = static_cast<int>(ceil(t / delta)) - 1;
  if (j < 0) j += n;
  if (j >= n) j -= n;
  return j;
}

// Pool of `cap` photon times per wave: mean of 64 periods' photons plus ten
// standard deviations (host).
__device__ inline double* pool_segment(double* pool, int cap, int want, int lane, int* room) {
  const int off = wave_exclusive_sum(want, lane);
  *room = min(want, max(cap - off, 0));
  return pool + off;
}

// Grid: pixels x chain_blocks blocks, pixel-major (block b: pixel b /
// chain_blocks), so that consecutive blocks, which the dispatcher deals to
// the XCDs in turn, spread every pixel over all of them (a 2D grid with the
// pixel as its x would pin pixel x to XCD x mod 8 whenever the pixel count is
// a multiple of 8, and the XCD with the brightest pixels would set the time).
// Block = WPB wavefronts of 64 / L chains each, all of one pixel.
// Chain q of a pixel is segment q mod K of run q / K: periods
// [seg len (q mod K), min(seg len (q mod K + 1), cycles)), started armed; with
// K > 1 its last rearm time goes to spec_end.
// LDS: per wavefront, a pool of `cap` photon times shared by its 64 periods
// of a chunk (each lane owns a contiguous segment, placed by a prefix sum of
// its Poisson counts, sorted); per wavefront, for groups that share the
// search, for each photon the last registration of the chain that starts
// with it (uint16, same offsets); then the pixel's histogram (n uint32),
// shared by the block's wavefronts and added atomically to HBM at the end.
__global__ __launch_bounds__(BT * WPB) void k_mc(const PixelMeta* __restrict__ metas, int runs, int64_t cycles,
                                           int64_t burn, uint64_t seed, int L, int cap, int K, int64_t seg_len,
                                           int chain_blocks, uint32_t* __restrict__ hist,
                                           uint32_t* __restrict__ overflow, double* __restrict__ spec_end) {
  extern __shared__ double lds_d[];
  __shared__ double cdf_s[KMAX], cdf_b[KMAX];
  const int wid = static_cast<int>(threadIdx.x) / BT, lane = static_cast<int>(threadIdx.x) % BT;
  double* pool = lds_d + wid * cap;
  // jend (uint16 per pool slot) only for groups that share the search
  uint16_t* jend = reinterpret_cast<uint16_t*>(lds_d + WPB * cap) + wid * cap;
  uint32_t* h = reinterpret_cast<uint32_t*>(lds_d + WPB * cap) + (L >= kCoopMin ? (WPB * cap + 1) / 2 : 0);
  const int pix = static_cast<int>(blockIdx.x / chain_blocks), cb = static_cast<int>(blockIdx.x % chain_blocks);
  const PixelMeta m = metas[pix];
  const int n = m.n;
  for (int j = threadIdx.x; j < n; j += BT * WPB) h[j] = 0u;
  if (threadIdx.x == 0) poisson_cdf(m.S, m.e_s, cdf_s);
  if (threadIdx.x == 1) poisson_cdf(m.B, m.e_b, cdf_b);
  __syncthreads();
  const int k_in = lane % L, base_lane = lane - k_in;
  const int64_t chain = (static_cast<int64_t>(cb) * WPB + wid) * (BT / L) + lane / L;
  const int run = static_cast<int>(chain / K), sgm = static_cast<int>(chain % K);
  const bool run_ok = run < runs;
  const int64_t seg_begin = sgm * seg_len, seg_end = min(seg_begin + seg_len, cycles);
  const double delta = m.t_r / n;
  bool over = false;
  double a = 0.0;  // rearm time of this lane's chain, relative to the chunk's next period
  for (int64_t c0 = 0; c0 < seg_len; c0 += L) {
    const int64_t c = seg_begin + c0 + k_in;
    const bool mine = run_ok && c < seg_end;
    const Draws st = period_stream(seed, c, run, m);
    int ns = 0, nb = 0;
    if (mine) period_counts(st, cdf_s, cdf_b, ns, nb);
    const int off = wave_exclusive_sum(ns + nb, lane);
    const int room = min(ns + nb, max(cap - off, 0));
    double* seg = pool + off;
    int cnt = 0;
    if (mine) {
      cnt = period_photons(m, st, ns, nb, seg, room, &over);
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
          atomicAdd(&h[bin_of(t, delta, n)], 1u);
        }
      }
    }
  }
  // every lane of a group holds the chain's final rearm time
  if (K > 1 && run_ok && k_in == 0) spec_end[(static_cast<int64_t>(pix) * runs + run) * K + sgm] = a;
  if (over) atomicOr(&overflow[m.index], 1u);
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += BT * WPB)
    if (h[j]) atomicAdd(&hist[m.pi_off + j], h[j]);
}

// Per-lane state of a pair walk: trajectories 1 and 2 (rearm times a1, a2)
// through periods [c, c_end) of one run.
struct PairWalk {
  double a1, a2;
  int64_t c, c_end;
  bool on;
};

// One period of every active pair walk of the wave (all lanes call it): the
// period's photons, trajectory 1's registrations added and trajectory 2's
// removed (periods >= burn; a photon both register changes nothing), then
// the next period.  A walk ends once a1 == a2 at a period start (coupled: the
// trajectories agree from there on) or at c_end.
__device__ inline void pair_period(PairWalk& w, const PixelMeta& m, int run, uint64_t seed, int64_t burn,
                                   const double* cdf_s, const double* cdf_b, double* pool, int cap, int lane,
                                   uint32_t* __restrict__ hist, bool* over) {
  const Draws st = period_stream(seed, w.c, run, m);
  int ns = 0, nb = 0;
  if (w.on) period_counts(st, cdf_s, cdf_b, ns, nb);
  int room;
  double* seg = pool_segment(pool, cap, ns + nb, lane, &room);
  if (w.on) {
    const int cnt = period_photons(m, st, ns, nb, seg, room, over);
    const double delta = m.t_r / m.n;
    const bool counted = w.c >= burn;
    for (int x = 0; x < cnt; ++x) {
      const double t = seg[x];
      const bool r1 = t >= w.a1, r2 = t >= w.a2;
      if (r1) w.a1 = t + m.t_d;
      if (r2) w.a2 = t + m.t_d;
      if (counted && r1 != r2) atomicAdd(&hist[m.pi_off + bin_of(t, delta, m.n)], r1 ? 1u : 0xFFFFFFFFu);
    }
    w.a1 = fmax(w.a1 - m.t_r, 0.0);
    w.a2 = fmax(w.a2 - m.t_r, 0.0);
    w.c += 1;
    if (w.a1 == w.a2 || w.c == w.c_end) w.on = false;
  }
}

// Repair of a segmented simulation (see the top of this file).  Grid:
// pixels x item_blocks blocks, pixel-major as in k_mc; one wave per block,
// one lane per item.
// CHAIN = false: item = (run, segment s >= 1).  Walk s from the speculative
// end of s - 1 (trajectory 1) beside the armed start (trajectory 2); record
// whether they coupled and trajectory 1's end.
// CHAIN = true: item = run.  Follow the true rearm time along the segments;
// where a segment's true start differs from the start the first pass
// assumed, walk it again from the true start (1) beside the assumed one (2).
// True end of segment s: its speculative end if the assumed trajectory
// coupled with the armed one, else that trajectory's recorded end, unless
// the true trajectory never met the assumed one (then its own end).
template <bool CHAIN>
__global__ __launch_bounds__(BT) void k_mc_repair(const PixelMeta* __restrict__ metas, int runs, int64_t cycles,
                                                  int64_t burn, uint64_t seed, int cap, int K, int64_t seg_len,
                                                  int item_blocks, uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ overflow, const double* __restrict__ spec_end,
                                                  double* __restrict__ end1, int32_t* __restrict__ coupled) {
  extern __shared__ double lds_d[];
  __shared__ double cdf_s[KMAX], cdf_b[KMAX];
  const int pix = static_cast<int>(blockIdx.x / item_blocks), ib = static_cast<int>(blockIdx.x % item_blocks);
  const PixelMeta m = metas[pix];
  const int lane = threadIdx.x;
  if (lane == 0) poisson_cdf(m.S, m.e_s, cdf_s);
  if (lane == 1) poisson_cdf(m.B, m.e_b, cdf_b);
  __syncthreads();
  const int64_t item = static_cast<int64_t>(ib) * BT + lane;
  const int64_t items = CHAIN ? runs : static_cast<int64_t>(runs) * (K - 1);
  const bool ok = item < items;
  const int run = static_cast<int>(CHAIN ? item : item / (K - 1));
  const int64_t base = (static_cast<int64_t>(pix) * runs + run) * K;
  bool over = false;
  PairWalk w{0.0, 0.0, 0, 0, false};
  int sgm = CHAIN ? 1 : static_cast<int>(item % (K - 1)) + 1;
  double true_prev = 0.0;  // CHAIN: true rearm time at the start of segment sgm
  bool alive = ok;
  if (ok) {
    if (CHAIN) {
      true_prev = spec_end[base];  // segment 0 starts armed: its first pass was exact
    } else {
      w.a1 = spec_end[base + sgm - 1];
      w.a2 = 0.0;
      w.c = sgm * seg_len;
      w.c_end = min(w.c + seg_len, cycles);
      w.on = w.a1 != w.a2;
    }
  }
  for (;;) {
    if (CHAIN && alive && !w.on) {
      // past the segments whose assumed start was the true one
      while (sgm < K) {
        const double assumed = spec_end[base + sgm - 1];
        if (true_prev != assumed) break;
        true_prev = coupled[base + sgm] ? spec_end[base + sgm] : end1[base + sgm];
        ++sgm;
      }
      if (sgm == K) {
        alive = false;
      } else {
        w.a1 = true_prev;
        w.a2 = spec_end[base + sgm - 1];
        w.c = sgm * seg_len;
        w.c_end = min(w.c + seg_len, cycles);
        w.on = true;
      }
    }
    if (!__any(w.on)) break;
    const bool was_on = w.on;
    pair_period(w, m, run, seed, burn, cdf_s, cdf_b, lds_d, cap, lane, hist, &over);
    if (was_on && !w.on) {
      if (CHAIN) {
        true_prev = w.a1 == w.a2 ? (coupled[base + sgm] ? spec_end[base + sgm] : end1[base + sgm]) : w.a1;
        ++sgm;
      } else {
        alive = false;
      }
    }
  }
  if (!CHAIN && ok) {
    coupled[base + sgm] = w.a1 == w.a2 ? 1 : 0;
    end1[base + sgm] = w.a1;
  }
  if (over) atomicOr(&overflow[m.index], 1u);
}

}  // namespace mc
}  // namespace dtm

using namespace dtm;

namespace {

// Segments per run (K, after dropping empty ones) and periods per segment.
// segments_per_run 0 picks about 2^18 chains in all (measured on the paper's
// sweeps: 2^17 to 2^19 chains run within 5 % of each other) with segments of
// at least 256 periods (their repair walks, a few periods each, stay a small
// share).
void mc_segments(const dtm_plan* plan, int32_t runs_per_pixel, int64_t cycles, int32_t segments_per_run,
                 int64_t* K_out, int64_t* seg_len_out) {
  const double runs_total = static_cast<double>(plan->n_pixels) * runs_per_pixel;
  int64_t K = segments_per_run;
  if (K == 0) {
    K = static_cast<int64_t>(std::ceil(262144.0 / runs_total));
    K = std::max<int64_t>(1, std::min<int64_t>(K, cycles / 256));
  }
  const int64_t seg_len = (cycles + K - 1) / K;
  *K_out = (cycles + seg_len - 1) / seg_len;
  *seg_len_out = seg_len;
}

size_t mc_state_bytes(const dtm_plan* plan, int32_t runs_per_pixel, int64_t K) {
  if (K <= 1) return 0;
  const size_t chains = static_cast<size_t>(plan->n_pixels) * static_cast<size_t>(runs_per_pixel) *
                        static_cast<size_t>(K);
  return chains * (2 * sizeof(double) + sizeof(int32_t));
}

}  // namespace

extern "C" size_t dtm_mc_scratch_bytes(const dtm_plan* plan, int32_t runs_per_pixel, int64_t cycles,
                                       int32_t segments_per_run) {
  if (!plan || runs_per_pixel < 1 || cycles < 1 || segments_per_run < 0 || segments_per_run > cycles) return 0;
  int64_t K, seg_len;
  mc_segments(plan, runs_per_pixel, cycles, segments_per_run, &K, &seg_len);
  return mc_state_bytes(plan, runs_per_pixel, K);
}

extern "C" int dtm_mc_histograms(const dtm_plan* plan, int32_t runs_per_pixel, int64_t cycles,
                                 int64_t burn_cycles, uint64_t seed, int32_t lanes_per_run,
                                 int32_t segments_per_run, uint32_t* hist_packed_dev, uint32_t* overflow_dev,
                                 void* scratch_dev, size_t scratch_bytes, dtm_stream_t stream) {
  if (!plan || !plan->ws || !hist_packed_dev || !overflow_dev) return DTM_EINVAL;
  if (runs_per_pixel < 1 || runs_per_pixel > 65535 || cycles < 1 || cycles > 0xFFFFFFFFll ||
      burn_cycles < 0 || burn_cycles >= cycles)
    return DTM_EINVAL;
  if (static_cast<double>(runs_per_pixel) * static_cast<double>(cycles - burn_cycles) >= 67108864.0)
    return DTM_EINVAL;
  if (lanes_per_run < 0 || lanes_per_run > mc::BT || (lanes_per_run & (lanes_per_run - 1)))
    return DTM_EINVAL;
  if (segments_per_run < 0 || segments_per_run > cycles) return DTM_EINVAL;
  if (plan->max_n > 16384) return DTM_ENOTSUP;
  for (const PixelMeta& m : plan->meta)
    if (m.S + m.B > 24.0) return DTM_ENOTSUP;
  int64_t K, seg_len;
  mc_segments(plan, runs_per_pixel, cycles, segments_per_run, &K, &seg_len);
  const double runs_total = static_cast<double>(plan->n_pixels) * runs_per_pixel;
  if (runs_total * static_cast<double>(K) > 134217728.0) return DTM_EINVAL;
  const size_t state_bytes = mc_state_bytes(plan, runs_per_pixel, K);
  if (state_bytes > 0 && (!scratch_dev || (reinterpret_cast<uintptr_t>(scratch_dev) & 255u))) return DTM_EINVAL;
  if (scratch_bytes < state_bytes) return DTM_ENOSPACE;
  int L = lanes_per_run;
  if (L == 0) {
    // At least 4 lanes per chain, more until the chains give about one and a
    // half waves to each SIMD of the 256 CUs (measured: the longer hand-over
    // chain of a larger group costs less than an idle SIMD).
    const double chains = runs_total * static_cast<double>(K);
    L = 4;
    while (L < mc::BT && chains * L < 256.0 * 4 * 64 * 1.5) L *= 2;
  }
  const int per_block = mc::WPB * (mc::BT / L);
  const int64_t chain_blocks = (static_cast<int64_t>(runs_per_pixel) * K + per_block - 1) / per_block;
  const int64_t fix_blocks = (static_cast<int64_t>(runs_per_pixel) * (K - 1) + mc::BT - 1) / mc::BT;
  const int64_t chain_blocks_b = (static_cast<int64_t>(runs_per_pixel) + mc::BT - 1) / mc::BT;
  if (static_cast<double>(plan->n_pixels) * static_cast<double>(chain_blocks) >= 2147483647.0 ||
      static_cast<double>(plan->n_pixels) * static_cast<double>(fix_blocks) >= 2147483647.0)
    return DTM_EINVAL;
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
  const size_t lds = sizeof(double) * static_cast<size_t>(mc::WPB * cap) +
                    (L >= mc::kCoopMin ? sizeof(uint32_t) * static_cast<size_t>((mc::WPB * cap + 1) / 2) : 0) +
                    sizeof(uint32_t) * static_cast<size_t>(plan->max_n);
  if (lds > 160 * 1024) return DTM_ENOTSUP;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(mc::k_mc), hipFuncAttributeMaxDynamicSharedMemorySize,
                          static_cast<int>(lds)) != hipSuccess)
    return DTM_EHIP;
  // segment states: speculative ends, repaired ends, coupled flags
  const size_t chains_total = static_cast<size_t>(runs_total) * static_cast<size_t>(K);
  double* spec_end = K > 1 ? static_cast<double*>(scratch_dev) : nullptr;
  double* end1 = K > 1 ? spec_end + chains_total : nullptr;
  int32_t* coupled = K > 1 ? reinterpret_cast<int32_t*>(end1 + chains_total) : nullptr;
  const size_t total = plan->pi_elems;
  hipLaunchKernelGGL(mc::k_zero, dim3(static_cast<unsigned>((total + mc::BT - 1) / mc::BT)), dim3(mc::BT), 0, st,
                     hist_packed_dev, total);
  hipLaunchKernelGGL(mc::k_mc, dim3(static_cast<unsigned>(plan->n_pixels * chain_blocks)), dim3(mc::BT * mc::WPB), lds, st,
                     metas, runs_per_pixel, cycles, burn_cycles, seed, L, cap, static_cast<int>(K), seg_len,
                     static_cast<int>(chain_blocks), hist_packed_dev, overflow_dev, spec_end);
  if (K > 1) {
    const size_t lds_fix = sizeof(double) * static_cast<size_t>(cap);
    hipLaunchKernelGGL(mc::k_mc_repair<false>, dim3(static_cast<unsigned>(plan->n_pixels * fix_blocks)),
                       dim3(mc::BT), lds_fix, st, metas, runs_per_pixel, cycles, burn_cycles, seed, cap,
                       static_cast<int>(K), seg_len, static_cast<int>(fix_blocks), hist_packed_dev, overflow_dev,
                       spec_end, end1, coupled);
    hipLaunchKernelGGL(mc::k_mc_repair<true>, dim3(static_cast<unsigned>(plan->n_pixels * chain_blocks_b)),
                       dim3(mc::BT), lds_fix, st, metas, runs_per_pixel, cycles, burn_cycles, seed, cap,
                       static_cast<int>(K), seg_len, static_cast<int>(chain_blocks_b), hist_packed_dev,
                       overflow_dev, spec_end, end1, coupled);
  }
  return hipGetLastError() == hipSuccess ? DTM_OK : DTM_EHIP;
}
