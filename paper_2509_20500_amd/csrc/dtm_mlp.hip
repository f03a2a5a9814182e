// Learned warm start for power iteration: a 5 -> 256 -> 256 -> 1024 MLP with
// GELU activations and a softmax output, trained on stationary PDFs produced
// by the solver itself.  GEMMs run on the MFMA units in bfloat16 with float32
// accumulation; activations, softmax, loss, gradients of biases and the Adam
// update are float32.  Float32 master weights, bfloat16 copies for the GEMMs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "dtm.h"
#include "dtm_internal.h"

namespace dtm {
namespace mlp {

constexpr int IN = DTM_MLP_IN;
constexpr int INP = DTM_MLP_IN_PAD;
constexpr int H = DTM_MLP_HIDDEN;
constexpr int OUT = DTM_MLP_OUT;

typedef uint16_t bf16;
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline float bf2f(bf16 h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }
// float -> bfloat16, round to nearest even (finite inputs).
__device__ inline bf16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<bf16>(u >> 16);
}

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
         x * 0.39894228040143268f * expf(-0.5f * x * x);
}

enum Epi { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2 };

// C[M x N] = op(A)[M x K] op(B)[K x N] with op(A)[i][k] = TA ? A[k*lda+i] :
// A[i*lda+k] and op(B)[k][j] = TB ? B[j*ldb+k] : B[k*ldb+j].  A 64 x 64 tile
// per block of 4 wavefronts, each wavefront a 32 x 32 quarter computed as
// 2 x 2 v_mfma_f32_16x16x32_bf16 tiles; K advances by GK = 64 through LDS
// (two MFMA steps of 32 per stage, in k order).
// Lane layout of the 16x16x32 instruction: lane l supplies A[l%16][8(l/16)+r]
// and B[8(l/16)+r][l%16] (r = 0..7) and receives D[4(l/16)+r][l%16]
// (r = 0..3).
// Split K (gridDim.z > 1): block z covers k in [z kc, (z + 1) kc) and
// writes its partial product to C + z * M * ldc; k_sum_splits adds the
// partials in z order.
// Out-of-range elements load as zero and are not stored.
constexpr int GK = 64;
constexpr int LDS_PITCH = GK + 8;  // 144-byte rows: every 8-element k run is one aligned 16-byte LDS read

typedef uint16_t bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 mfma_bf16x8 __attribute__((ext_vector_type(8)));

// Thread tid's share of a 64 x GK operand tile T[r][kk] = op(X)[o + r][k0 + kk]:
// the 16 elements idx = 16 tid + e.  ALONG_R: X is stored k-major
// (X[k * ld + i]), the run goes along r; otherwise X[i * ld + k] and the
// run goes along kk.  Out-of-range elements are zero.
template <bool ALONG_R>
__device__ inline void load_run(const bf16* __restrict__ X, int ld, int rows, int K, int o, int k0, int tid,
                                bf16 (&T)[64][LDS_PITCH]) {
  const int idx0 = tid * 16;
  const int r0 = ALONG_R ? idx0 % 64 : idx0 / GK, kk0 = ALONG_R ? idx0 / 64 : idx0 % GK;
  const int gi0 = o + r0, gk0 = k0 + kk0;
  const bf16* src = ALONG_R ? X + static_cast<int64_t>(gk0) * ld + gi0 : X + static_cast<int64_t>(gi0) * ld + gk0;
  const bool full = ALONG_R ? (gk0 < K && gi0 + 16 <= rows) : (gi0 < rows && gk0 + 16 <= K);
  bf16 v[16];
  if (full && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(src);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(src + 8);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      v[e] = a[e];
      v[8 + e] = b[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int gi = ALONG_R ? gi0 + e : gi0, gk = ALONG_R ? gk0 : gk0 + e;
      v[e] = (gi < rows && gk < K) ? X[ALONG_R ? static_cast<int64_t>(gk) * ld + gi
                                               : static_cast<int64_t>(gi) * ld + gk]
                                   : static_cast<bf16>(0);
    }
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) T[ALONG_R ? r0 + e : r0][ALONG_R ? kk0 : kk0 + e] = v[e];
}

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const bf16* __restrict__ A,
                                              int lda, const bf16* __restrict__ B, int ldb,
                                              float* __restrict__ C, int ldc,
                                              const float* __restrict__ bias,
                                              bf16* __restrict__ Hout, int ldh, int kc) {
  __shared__ __align__(16) bf16 As[64][LDS_PITCH];
  __shared__ __align__(16) bf16 Bs[64][LDS_PITCH];  // transposed: Bs[j][k]
  const int tid = threadIdx.x;
  const int lane = tid % 64, wave = tid / 64;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int wi = (wave / 2) * 32, wj = (wave % 2) * 32;
  const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
  C += static_cast<int64_t>(blockIdx.z) * M * ldc;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += GK) {
    // 64 x GK tiles: thread t loads 16 consecutive elements of each along
    // the operand's contiguous dimension (k for a row-major A or a
    // transposed B, the row or column index otherwise): two 16-byte loads
    // when the run is in range and aligned, else element by element
    load_run<TA>(A, lda, M, ke, i0, k0, tid, As);
    load_run<!TB>(B, ldb, N, ke, j0, k0, tid, Bs);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK; ks += 32) {
      const int kq = ks + 8 * (lane / 16);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int ra = wi + a * 16 + lane % 16;
        const mfma_bf16x8 fa = *reinterpret_cast<const mfma_bf16x8*>(&As[ra][kq]);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int cb = wj + b * 16 + lane % 16;
          const mfma_bf16x8 fb = *reinterpret_cast<const mfma_bf16x8*>(&Bs[cb][kq]);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[a][b], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wi + a * 16 + 4 * (lane / 16) + r;
        const int gj = j0 + wj + b * 16 + lane % 16;
        if (gi >= M || gj >= N) continue;
        float v = acc[a][b][r];
        if (EPI != EPI_STORE) v += bias[gj];
        C[static_cast<int64_t>(gi) * ldc + gj] = v;
        if (EPI == EPI_BIAS_GELU) Hout[static_cast<int64_t>(gi) * ldh + gj] = f2bf(gelu(v));
      }
}

// C[i][j] = sum over z of part[z][i][j] (M x N, row-major, dense), in z order.
__global__ void k_sum_splits(const float* __restrict__ part, int splits, int64_t mn, float* __restrict__ C) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= mn) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[static_cast<int64_t>(z) * mn + idx];
  C[idx] = s;
}

// Features of a scene, fixed affine maps onto about [-1, 1]:
//   2 u, sigma / 1 ns, 2 (ln S - ln 0.05) / ln 100 - 1,
//   2 (ln B - ln 0.01) / ln 100 - 1, (t_d mod t_r) / t_r,
// with the pulse bin k = floor(tau / (t_r / OUT)) (written to shift) and u
// the pulse's offset from that bin's centre, in [-1/2, 1/2).  The output
// layer works in the frame of bin k (k_softmax_xent rotates it), so the
// pulse's absolute position is not a feature.
__global__ void k_features(const dtm_scene* __restrict__ scenes, int n, float* __restrict__ feat,
                           int32_t* __restrict__ shift) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const dtm_scene s = scenes[p];
  const double l100 = log(100.0);
  const double pos = s.pulse_center_ns / (s.period_ns / OUT);
  const double k = floor(pos);
  feat[p * IN + 0] = static_cast<float>(2.0 * (pos - k - 0.5));
  if (shift) shift[p] = static_cast<int32_t>(k);
  feat[p * IN + 1] = static_cast<float>(s.pulse_sigma_ns);
  feat[p * IN + 2] = static_cast<float>(2.0 * (log(fmax(s.signal_flux, 1e-30)) - log(0.05)) / l100 - 1.0);
  feat[p * IN + 3] = static_cast<float>(2.0 * (log(fmax(s.background_flux, 1e-30)) - log(0.01)) / l100 - 1.0);
  feat[p * IN + 4] = static_cast<float>(fmod(s.dead_time_ns, s.period_ns) / s.period_ns);
}

// Prior logits of the warm start: log(lambda_j / sum_k lambda_k) at the OUT
// bin centres s_j = (j + 1/2) t_r / OUT of each scene, lambda of
// Eq. (arrival_flux) (the flux start of the solver, the stationary vector
// without dead time).  Float64 in the log domain (a Gaussian far from its
// centre would underflow as a flux), stored as float32.  One block of 256
// threads per scene.
__global__ __launch_bounds__(256) void k_flux_prior(const dtm_scene* __restrict__ scenes, float* __restrict__ prior) {
  __shared__ double red[4];
  const dtm_scene s = scenes[blockIdx.x];
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  const double delta = s.period_ns / OUT, is = 1.0 / s.pulse_sigma_ns;
  const double la = s.signal_flux > 0.0 ? log(s.signal_flux * 0.39894228040143267794 * is) : -INFINITY;
  const double lb = s.background_flux > 0.0 ? log(s.background_flux / s.period_ns) : -INFINITY;
  double lv[4], mx = -INFINITY;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double z = ((tid + 256 * r + 0.5) * delta - s.pulse_center_ns) * is;
    const double a = la - 0.5 * z * z;
    const double hi = fmax(a, lb), lo = fmin(a, lb);
    lv[r] = hi == -INFINITY ? -INFINITY : hi + log1p(exp(lo - hi));
    mx = fmax(mx, lv[r]);
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) red[w] = mx;
  __syncthreads();
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  double sum = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) sum += exp(lv[r] - mx);
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if (lane == 0) red[w] = sum;
  __syncthreads();
  const double lse = mx + log((red[0] + red[1]) + (red[2] + red[3]));
#pragma unroll
  for (int r = 0; r < 4; ++r)
    prior[static_cast<int64_t>(blockIdx.x) * OUT + tid + 256 * r] = static_cast<float>(lv[r] - lse);
}

// X0 (bfloat16, rows padded to INP columns with zeros).
// X0 row i = the features of row rows[i] (row i without rows).
__global__ void k_pack_input(const float* __restrict__ feat, const int32_t* __restrict__ rows, int batch,
                             bf16* __restrict__ x0) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= batch * INP) return;
  const int i = idx / INP, k = idx % INP;
  const int64_t r = rows ? rows[i] : i;
  x0[idx] = k < IN ? f2bf(feat[r * IN + k]) : static_cast<bf16>(0);
}

// Row-wise softmax of the logits, rotated by the row's pulse bin k (bin j
// takes logit (j - k) mod OUT; k = 0 without shift), plus the prior logits
// (when given); optionally cross-entropy against a target distribution with
// its gradient dZ = (q - target) / batch written back at the rotated
// positions (float32 and bfloat16; the prior is a constant, so the gradient
// is the same).  The prior, pulse bin and target of batch row i are those
// of row rows[i] (row i without rows).  One block of 256 threads per row of
// OUT = 1024 logits.
__global__ __launch_bounds__(256) void k_softmax_xent(const float* __restrict__ z, int batch,
                                                      const float* __restrict__ prior,
                                                      const int32_t* __restrict__ shift,
                                                      const float* __restrict__ target,
                                                      const int32_t* __restrict__ rows,
                                                      float* __restrict__ q_out,
                                                      float* __restrict__ dz, bf16* __restrict__ dzb,
                                                      float* __restrict__ loss) {
  __shared__ float red[4];
  const int i = blockIdx.x;
  const int64_t src = rows ? rows[i] : i;
  const float* zr = z + static_cast<int64_t>(i) * OUT;
  const int k = shift ? shift[src] : 0;
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  float v[4];
  float mx = -INFINITY;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    v[r] = zr[(tid + 256 * r - k) & (OUT - 1)];
    if (prior) v[r] += prior[src * OUT + tid + 256 * r];
    mx = fmaxf(mx, v[r]);
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) red[w] = mx;
  __syncthreads();
  mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  __syncthreads();
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    v[r] = expf(v[r] - mx);
    s += v[r];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) red[w] = s;
  __syncthreads();
  s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  const float lse = mx + logf(s);
  float l = 0.f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int j = tid + 256 * r;
    const int m = (j - k) & (OUT - 1);
    const float q = v[r] / s;
    const float zj = zr[m] + (prior ? prior[src * OUT + j] : 0.f);
    if (q_out) q_out[static_cast<int64_t>(i) * OUT + j] = q;
    if (target) {
      const float t = target[src * OUT + j];
      l -= t * (zj - lse);
      const float g = (q - t) / batch;
      dz[static_cast<int64_t>(i) * OUT + m] = g;
      dzb[static_cast<int64_t>(i) * OUT + m] = f2bf(g);
    }
  }
  if (target) {
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
    if (lane == 0) red[w] = l;
    __syncthreads();
    if (tid == 0) loss[i] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// dA = dH * gelu'(A) (float32 and bfloat16).
__global__ void k_gelu_back(const float* __restrict__ dh, const float* __restrict__ a, int n,
                            float* __restrict__ da, bf16* __restrict__ dab) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const float g = dh[idx] * gelu_grad(a[idx]);
  da[idx] = g;
  dab[idx] = f2bf(g);
}

// db[j] = sum_i d[i][j] in a fixed order: a block owns BG_COLS columns; its
// BG_GROUPS thread groups each add one contiguous chunk of rows in row
// order (eight loads issued ahead of their adds), and the chunk sums are
// then added in chunk order.
constexpr int BG_COLS = 16;
constexpr int BG_THREADS = 1024;
constexpr int BG_GROUPS = BG_THREADS / BG_COLS;

__global__ __launch_bounds__(BG_THREADS) void k_bias_grad(const float* __restrict__ d, int rows, int cols,
                                                          float* __restrict__ db) {
  __shared__ float part[BG_GROUPS][BG_COLS];
  const int c = threadIdx.x % BG_COLS, g = threadIdx.x / BG_COLS;
  const int j = blockIdx.x * BG_COLS + c;
  const int chunk = (rows + BG_GROUPS - 1) / BG_GROUPS;
  const int i0 = min(g * chunk, rows), i1 = min(i0 + chunk, rows);
  float s = 0.f;
  if (j < cols) {
    const float* col = d + j;
    int i = i0;
    for (; i + 8 <= i1; i += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = col[static_cast<int64_t>(i + u) * cols];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; i < i1; ++i) s += col[static_cast<int64_t>(i) * cols];
  }
  part[g][c] = s;
  __syncthreads();
  if (g == 0 && j < cols) {
    float t = 0.f;
    for (int q = 0; q < BG_GROUPS; ++q) t += part[q][c];
    db[j] = t;
  }
}

// Adam on the flat float32 parameters; refreshes their bfloat16 copies.
__global__ void k_adam(float* __restrict__ w, bf16* __restrict__ wb, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= n) return;
  const float gi = g[idx];
  const float mi = b1 * m[idx] + (1.f - b1) * gi;
  const float vi = b2 * v[idx] + (1.f - b2) * gi * gi;
  m[idx] = mi;
  v[idx] = vi;
  const float wi = w[idx] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[idx] = wi;
  wb[idx] = f2bf(wi);
}

__global__ void k_to_bf16(const float* __restrict__ w, bf16* __restrict__ wb, int64_t n) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx < n) wb[idx] = f2bf(w[idx]);
}

// ---- layout -----------------------------------------------------------------

struct Ptrs {
  float *p, *g, *m, *v;
  bf16* pb;
  float *w1, *b1, *w2, *b2, *w3, *b3;
  float *gw1, *gb1, *gw2, *gb2, *gw3, *gb3;
  bf16 *w1b, *w2b, *w3b;
  bf16* x0;
  float *a1, *a2, *z, *q, *dz, *dh2, *da2, *dh1, *da1, *loss;
  bf16 *h1, *h2, *dzb, *da2b, *da1b;
  float* partial;
};

// Split of K (= the batch) for a weight-gradient GEMM with an M x N output:
// enough blocks to cover the chip's 256 CUs once (at most 16 splits), chunks
// of at least GK.  Returns the chunk length kc (a multiple of GK); the split
// count is ceil(K / kc).
int grad_chunk(int M, int N, int K) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int s = std::max(1, std::min(16, 256 / tiles));
  s = std::min(s, std::max(1, K / GK));
  return ((K + s - 1) / s + GK - 1) / GK * GK;
}
int64_t grad_partial_floats(int M, int N, int K) {
  const int kc = grad_chunk(M, N, K);
  const int s = (K + kc - 1) / kc;
  return s > 1 ? static_cast<int64_t>(s) * M * N : 0;
}
// Largest partial buffer of the three weight gradients at this batch size
// (the split count never falls as the batch grows).
int64_t partial_floats(int32_t max_batch) {
  return std::max(grad_partial_floats(H, OUT, max_batch),
                  std::max(grad_partial_floats(H, H, max_batch), grad_partial_floats(INP, H, max_batch)));
}

void layout(int32_t max_batch, dtm_mlp_layout* L) {
  const int64_t B = max_batch;
  L->off_w1 = 0;
  L->off_b1 = L->off_w1 + static_cast<int64_t>(INP) * H;
  L->off_w2 = L->off_b1 + H;
  L->off_b2 = L->off_w2 + static_cast<int64_t>(H) * H;
  L->off_w3 = L->off_b2 + H;
  L->off_b3 = L->off_w3 + static_cast<int64_t>(H) * OUT;
  L->n_params = L->off_b3 + OUT;
  L->max_batch = max_batch;
  L->reserved = 0;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t np = static_cast<size_t>(L->n_params);
  L->params = take(4 * np);
  L->params_bf16 = take(2 * np);
  L->grads = take(4 * np);
  L->adam_m = take(4 * np);
  L->adam_v = take(4 * np);
  // activations
  L->act = off;
  take(2 * B * INP);            // x0
  take(4 * B * H);              // a1
  take(2 * B * H);              // h1
  take(4 * B * H);              // a2
  take(2 * B * H);              // h2
  take(4 * B * OUT);            // z
  take(4 * B * OUT);            // q
  take(4 * B * OUT);            // dz
  take(2 * B * OUT);            // dzb
  take(4 * B * H);              // dh2
  take(4 * B * H);              // da2
  take(2 * B * H);              // da2b
  take(4 * B * H);              // dh1
  take(4 * B * H);              // da1
  take(2 * B * H);              // da1b
  take(4 * B);                  // loss
  // split-K partial products of the weight gradients
  L->partial = take(4 * partial_floats(max_batch));
  L->total = off;
}

Ptrs pointers(void* ws, int32_t max_batch) {
  dtm_mlp_layout L;
  layout(max_batch, &L);
  char* w = static_cast<char*>(ws);
  Ptrs P;
  P.p = reinterpret_cast<float*>(w + L.params);
  P.pb = reinterpret_cast<bf16*>(w + L.params_bf16);
  P.g = reinterpret_cast<float*>(w + L.grads);
  P.m = reinterpret_cast<float*>(w + L.adam_m);
  P.v = reinterpret_cast<float*>(w + L.adam_v);
  P.w1 = P.p + L.off_w1; P.b1 = P.p + L.off_b1; P.w2 = P.p + L.off_w2;
  P.b2 = P.p + L.off_b2; P.w3 = P.p + L.off_w3; P.b3 = P.p + L.off_b3;
  P.gw1 = P.g + L.off_w1; P.gb1 = P.g + L.off_b1; P.gw2 = P.g + L.off_w2;
  P.gb2 = P.g + L.off_b2; P.gw3 = P.g + L.off_w3; P.gb3 = P.g + L.off_b3;
  P.w1b = P.pb + L.off_w1; P.w2b = P.pb + L.off_w2; P.w3b = P.pb + L.off_w3;
  const int64_t B = max_batch;
  size_t off = L.act;
  auto take = [&](size_t bytes) {
    char* q = w + off;
    off = align256(off + bytes);
    return q;
  };
  P.x0 = reinterpret_cast<bf16*>(take(2 * B * INP));
  P.a1 = reinterpret_cast<float*>(take(4 * B * H));
  P.h1 = reinterpret_cast<bf16*>(take(2 * B * H));
  P.a2 = reinterpret_cast<float*>(take(4 * B * H));
  P.h2 = reinterpret_cast<bf16*>(take(2 * B * H));
  P.z = reinterpret_cast<float*>(take(4 * B * OUT));
  P.q = reinterpret_cast<float*>(take(4 * B * OUT));
  P.dz = reinterpret_cast<float*>(take(4 * B * OUT));
  P.dzb = reinterpret_cast<bf16*>(take(2 * B * OUT));
  P.dh2 = reinterpret_cast<float*>(take(4 * B * H));
  P.da2 = reinterpret_cast<float*>(take(4 * B * H));
  P.da2b = reinterpret_cast<bf16*>(take(2 * B * H));
  P.dh1 = reinterpret_cast<float*>(take(4 * B * H));
  P.da1 = reinterpret_cast<float*>(take(4 * B * H));
  P.da1b = reinterpret_cast<bf16*>(take(2 * B * H));
  P.loss = reinterpret_cast<float*>(take(4 * B));
  P.partial = reinterpret_cast<float*>(w + L.partial);
  return P;
}

template <bool TA, bool TB, int EPI>
void gemm(int M, int N, int K, const bf16* A, int lda, const bf16* B, int ldb, float* C, int ldc,
          const float* bias, bf16* Hout, int ldh, hipStream_t st) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc,
                     bias, Hout, ldh, K);
}

// Weight gradient C (M x N, dense) = A^T B with K = the batch, K split over
// blocks when the output alone has too few tiles to fill the chip; the
// partial products go to `part` and are added in split order (the result
// does not depend on timing).
void gemm_grad(int M, int N, int K, const bf16* A, int lda, const bf16* B, int ldb, float* C, float* part,
               hipStream_t st) {
  const int kc = grad_chunk(M, N, K);
  const int splits = (K + kc - 1) / kc;
  if (splits == 1) {
    gemm<true, false, EPI_STORE>(M, N, K, A, lda, B, ldb, C, N, nullptr, nullptr, 0, st);
    return;
  }
  dim3 grid((N + 63) / 64, (M + 63) / 64, splits);
  hipLaunchKernelGGL((k_gemm<true, false, EPI_STORE>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, part, N,
                     nullptr, nullptr, 0, kc);
  const int64_t mn = static_cast<int64_t>(M) * N;
  hipLaunchKernelGGL(k_sum_splits, dim3(static_cast<unsigned>((mn + 255) / 256)), dim3(256), 0, st, part, splits,
                     mn, C);
}

// Forward pass for `batch` rows of features; leaves every activation in the
// workspace.
void forward(const Ptrs& P, const float* feat, const int32_t* rows, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_input, dim3((batch * INP + 255) / 256), dim3(256), 0, st, feat, rows, batch, P.x0);
  gemm<false, false, EPI_BIAS_GELU>(batch, H, INP, P.x0, INP, P.w1b, H, P.a1, H, P.b1, P.h1, H, st);
  gemm<false, false, EPI_BIAS_GELU>(batch, H, H, P.h1, H, P.w2b, H, P.a2, H, P.b2, P.h2, H, st);
  gemm<false, false, EPI_BIAS>(batch, OUT, H, P.h2, H, P.w3b, OUT, P.z, OUT, P.b3, nullptr, 0, st);
}

}  // namespace mlp
}  // namespace dtm

using namespace dtm;
using namespace dtm::mlp;

namespace {
int ok_launch() { return hipGetLastError() == hipSuccess ? DTM_OK : DTM_EHIP; }
bool batch_ok(int32_t batch, int32_t max_batch) {
  return max_batch >= 1 && max_batch <= DTM_MLP_MAX_BATCH && batch >= 1 && batch <= max_batch;
}
}  // namespace

extern "C" {

int dtm_mlp_workspace_layout(int32_t max_batch, dtm_mlp_layout* out) {
  if (!out || max_batch < 1 || max_batch > DTM_MLP_MAX_BATCH) return DTM_EINVAL;
  layout(max_batch, out);
  return DTM_OK;
}

int dtm_mlp_features(const dtm_scene* scenes_dev, int32_t n, float* feat_dev, int32_t* shift_dev,
                     dtm_stream_t stream) {
  if (!scenes_dev || !feat_dev || n < 1) return DTM_EINVAL;
  hipLaunchKernelGGL(k_features, dim3((n + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(stream), scenes_dev, n, feat_dev, shift_dev);
  return ok_launch();
}

int dtm_mlp_sync_bf16(void* ws, int32_t max_batch, dtm_stream_t stream) {
  if (!ws || max_batch < 1 || max_batch > DTM_MLP_MAX_BATCH) return DTM_EINVAL;
  dtm_mlp_layout L;
  layout(max_batch, &L);
  const Ptrs P = pointers(ws, max_batch);
  hipLaunchKernelGGL(k_to_bf16, dim3(static_cast<unsigned>((L.n_params + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), P.p, P.pb, L.n_params);
  return ok_launch();
}

int dtm_mlp_flux_prior(const dtm_scene* scenes_dev, int32_t n, float* prior_dev, dtm_stream_t stream) {
  if (!scenes_dev || !prior_dev || n < 1) return DTM_EINVAL;
  hipLaunchKernelGGL(k_flux_prior, dim3(n), dim3(256), 0, static_cast<hipStream_t>(stream), scenes_dev,
                     prior_dev);
  return ok_launch();
}

int dtm_mlp_forward(void* ws, int32_t max_batch, const float* feat_dev, const float* prior_dev,
                    const int32_t* shift_dev, int32_t batch, float* probs_dev, dtm_stream_t stream) {
  if (!ws || !feat_dev || !probs_dev || !batch_ok(batch, max_batch)) return DTM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Ptrs P = pointers(ws, max_batch);
  forward(P, feat_dev, nullptr, batch, st);
  hipLaunchKernelGGL(k_softmax_xent, dim3(batch), dim3(256), 0, st, P.z, batch, prior_dev, shift_dev, nullptr,
                     nullptr, probs_dev, nullptr, nullptr, nullptr);
  return ok_launch();
}

int dtm_mlp_backward(void* ws, int32_t max_batch, const float* feat_dev, const float* prior_dev,
                     const int32_t* shift_dev, const float* target_dev, const int32_t* rows_dev, int32_t batch,
                     float* loss_dev, dtm_stream_t stream) {
  if (!ws || !feat_dev || !target_dev || !batch_ok(batch, max_batch)) return DTM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Ptrs P = pointers(ws, max_batch);
  forward(P, feat_dev, rows_dev, batch, st);
  hipLaunchKernelGGL(k_softmax_xent, dim3(batch), dim3(256), 0, st, P.z, batch, prior_dev, shift_dev, target_dev,
                     rows_dev, P.q, P.dz, P.dzb, loss_dev ? loss_dev : P.loss);
  // layer 3: dW3 = H2^T dZ, db3 = sum dZ, dH2 = dZ W3^T
  gemm_grad(H, OUT, batch, P.h2, H, P.dzb, OUT, P.gw3, P.partial, st);
  hipLaunchKernelGGL(k_bias_grad, dim3((OUT + BG_COLS - 1) / BG_COLS), dim3(BG_THREADS), 0, st, P.dz, batch, OUT,
                     P.gb3);
  gemm<false, true, EPI_STORE>(batch, H, OUT, P.dzb, OUT, P.w3b, OUT, P.dh2, H, nullptr, nullptr, 0, st);
  hipLaunchKernelGGL(k_gelu_back, dim3((batch * H + 255) / 256), dim3(256), 0, st, P.dh2, P.a2,
                     batch * H, P.da2, P.da2b);
  // layer 2
  gemm_grad(H, H, batch, P.h1, H, P.da2b, H, P.gw2, P.partial, st);
  hipLaunchKernelGGL(k_bias_grad, dim3((H + BG_COLS - 1) / BG_COLS), dim3(BG_THREADS), 0, st, P.da2, batch, H,
                     P.gb2);
  gemm<false, true, EPI_STORE>(batch, H, H, P.da2b, H, P.w2b, H, P.dh1, H, nullptr, nullptr, 0, st);
  hipLaunchKernelGGL(k_gelu_back, dim3((batch * H + 255) / 256), dim3(256), 0, st, P.dh1, P.a1,
                     batch * H, P.da1, P.da1b);
  // layer 1
  gemm_grad(INP, H, batch, P.x0, INP, P.da1b, H, P.gw1, P.partial, st);
  hipLaunchKernelGGL(k_bias_grad, dim3((H + BG_COLS - 1) / BG_COLS), dim3(BG_THREADS), 0, st, P.da1, batch, H,
                     P.gb1);
  return ok_launch();
}

int dtm_mlp_adam(void* ws, int32_t max_batch, float lr, float beta1, float beta2, float eps,
                 int32_t step, dtm_stream_t stream) {
  if (!ws || max_batch < 1 || max_batch > DTM_MLP_MAX_BATCH || step < 1) return DTM_EINVAL;
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return DTM_EINVAL;
  dtm_mlp_layout L;
  layout(max_batch, &L);
  const Ptrs P = pointers(ws, max_batch);
  const float c1 = 1.f - std::pow(beta1, static_cast<float>(step));
  const float c2 = 1.f - std::pow(beta2, static_cast<float>(step));
  hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((L.n_params + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), P.p, P.pb, P.g, P.m, P.v, L.n_params, lr, beta1,
                     beta2, eps, c1, c2);
  return ok_launch();
}

int dtm_mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const void* A_dev, int32_t lda, int32_t trans_a,
                      const void* B_dev, int32_t ldb, int32_t trans_b, float* C_dev, int32_t ldc,
                      dtm_stream_t stream) {
  if (M < 1 || N < 1 || K < 1 || !A_dev || !B_dev || !C_dev) return DTM_EINVAL;
  if (ldc < N || lda < (trans_a ? M : K) || ldb < (trans_b ? K : N)) return DTM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bf16* A = static_cast<const bf16*>(A_dev);
  const bf16* B = static_cast<const bf16*>(B_dev);
  if (!trans_a && !trans_b) gemm<false, false, EPI_STORE>(M, N, K, A, lda, B, ldb, C_dev, ldc, nullptr, nullptr, 0, st);
  else if (trans_a && !trans_b) gemm<true, false, EPI_STORE>(M, N, K, A, lda, B, ldb, C_dev, ldc, nullptr, nullptr, 0, st);
  else if (!trans_a && trans_b) gemm<false, true, EPI_STORE>(M, N, K, A, lda, B, ldb, C_dev, ldc, nullptr, nullptr, 0, st);
  else gemm<true, true, EPI_STORE>(M, N, K, A, lda, B, ldb, C_dev, ldc, nullptr, nullptr, 0, st);
  return ok_launch();
}

}  // extern "C"
