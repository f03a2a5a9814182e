// Bandwidth of the dense solver's memory access pattern without its
// arithmetic, for the benchmark's calibration: one launch in which every
// block writes its chunk (as the build launch writes one pixel's matrix),
// then one in which every block streams its chunk back `reads` times with
// nontemporal loads (the sweep launch).
//
// A measurement aid, not part of the method: it is built into its own
// library, libdtm_probe.so, which only the benchmark and its test load.
//
//   int dtm_stream_probe(void* buf_dev, size_t chunk_bytes, int32_t n_chunks,
//                        int32_t reads, float* sink_dev, void* stream);
//
// buf_dev holds n_chunks * chunk_bytes bytes (caller owned, overwritten);
// sink_dev is one float that is never written for these values.  chunk_bytes
// a positive multiple of 16, n_chunks >= 1, reads >= 0, else DTM_EINVAL
// (nothing launched); a failed launch gives DTM_EHIP.  Launch only.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dtm.h"

namespace dtm {
namespace probe {

constexpr int BT = 256;
constexpr int UNROLL = 8;
typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(BT) void k_probe_write(f4* __restrict__ buf, size_t chunk4) {
  f4* p = buf + static_cast<size_t>(blockIdx.x) * chunk4;
  for (size_t i = threadIdx.x; i < chunk4; i += BT)
    __builtin_nontemporal_store(f4{1.0f, 2.0f, 3.0f, static_cast<float>(i)}, p + i);
}

__global__ __launch_bounds__(BT) void k_probe_read(const f4* __restrict__ buf, size_t chunk4, int reads,
                                                   float* __restrict__ sink) {
  const f4* p = buf + static_cast<size_t>(blockIdx.x) * chunk4;
  float s = 0.0f;
  for (int r = 0; r < reads; ++r) {
    size_t i = threadIdx.x;
    for (; i + (UNROLL - 1) * BT < chunk4; i += UNROLL * BT) {
      f4 v[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) v[u] = __builtin_nontemporal_load(p + i + u * BT);
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) s += v[u][0] + v[u][3];
    }
    for (; i < chunk4; i += BT) {
      const f4 v = __builtin_nontemporal_load(p + i);
      s += v[0] + v[3];
    }
  }
  if (s == -1.0f) sink[0] = s;  // keeps the loads; never true for these values
}

}  // namespace probe
}  // namespace dtm

extern "C" int dtm_stream_probe(void* buf_dev, size_t chunk_bytes, int32_t n_chunks, int32_t reads,
                                float* sink_dev, dtm_stream_t stream) {
  if (!buf_dev || !sink_dev || n_chunks < 1 || reads < 0 || chunk_bytes < 16 || chunk_bytes % 16 != 0)
    return DTM_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  dtm::probe::f4* buf = static_cast<dtm::probe::f4*>(buf_dev);
  hipLaunchKernelGGL(dtm::probe::k_probe_write, dim3(n_chunks), dim3(dtm::probe::BT), 0, st, buf, chunk_bytes / 16);
  hipLaunchKernelGGL(dtm::probe::k_probe_read, dim3(n_chunks), dim3(dtm::probe::BT), 0, st, buf, chunk_bytes / 16,
                     reads, sink_dev);
  return hipGetLastError() == hipSuccess ? DTM_OK : DTM_EHIP;
}
