// Host-side checks of the library's planning code (dtm_host.cpp), built with
// the address and undefined-behaviour sanitizers by tests/test_host_sanitizers.py.
// No GPU: plans are created, queried and freed without being bound.  Exits 0
// when every expectation holds; the sanitizers abort on the first memory or
// UB error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <limits>
#include <random>
#include <vector>

#include "dtm.h"
#include "dtm_internal.h"

static int failures = 0;
#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "%s:%d: failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                   \
    }                                                               \
  } while (0)

static dtm_scene make(std::mt19937_64& g, int32_t n) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  dtm_scene s;
  s.period_ns = 50.0 + 150.0 * u(g);
  s.dead_time_ns = s.period_ns * 2.5 * u(g);
  s.pulse_center_ns = s.period_ns * u(g);
  s.pulse_sigma_ns = 0.1 + u(g);
  s.signal_flux = 10.0 * u(g);
  s.background_flux = 0.01 + 10.0 * u(g);
  s.n_bins = n;
  s.reserved = 0;
  return s;
}

static void destroy(dtm_plan* p) { delete p; }  // unbound: no streams or events to release

int main() {
  std::mt19937_64 g(20500);
  // scenes: valid ones validate, and the shift rules stay in range
  for (int t = 0; t < 20000; ++t) {
    const int32_t n = 2 + static_cast<int32_t>(g() % 65535);
    dtm_scene s = make(g, n);
    EXPECT(dtm_validate_scene(&s) == DTM_OK);
    int32_t l = -1;
    EXPECT(dtm_shift_bins(&s, &l) == DTM_OK && l >= 0 && l < n);
    for (int32_t f : {0, DTM_FLAG_SHIFT_NEAREST, DTM_FLAG_SHIFT_INTERP}) {
      double frac = -1.0;
      EXPECT(dtm_model_shift(&s, f, &l, &frac) == DTM_OK && l >= 0 && l < n && frac >= 0.0 && frac < 1.0);
    }
  }
  // invalid scenes are refused
  const double bad[] = {0.0, -1.0, std::numeric_limits<double>::quiet_NaN(),
                        std::numeric_limits<double>::infinity()};
  for (int field = 0; field < 6; ++field)
    for (double v : bad) {
      dtm_scene s = make(g, 1024);
      double* f[] = {&s.period_ns, &s.dead_time_ns, &s.pulse_center_ns, &s.pulse_sigma_ns, &s.signal_flux,
                     &s.background_flux};
      *f[field] = v;
      const int rc = dtm_validate_scene(&s);
      // t_d, S and B may be 0; tau may lie anywhere (the pulse is cut to the period)
      const bool ok = std::isfinite(v) && (field == 2 || (v == 0.0 && (field == 1 || field == 4 || field == 5)));
      EXPECT((rc == DTM_OK) == ok);
    }
  for (int32_t n : {-5, 0, 1, 65537, std::numeric_limits<int32_t>::max()}) {
    dtm_scene s = make(g, 2);
    s.n_bins = n;
    EXPECT(dtm_validate_scene(&s) == DTM_EINVAL);
  }
  for (int c = -8; c <= 2; ++c) EXPECT(dtm_status_string(c) != nullptr);
  for (int32_t n : {2, 3, 1000, 4096, 65536}) {
    EXPECT(dtm_workspace_bytes(n, DTM_F32) > 0 && dtm_workspace_bytes(n, DTM_F64) > 0);
  }
  // plans: random uneven batches, tiles and options, valid and invalid
  const int32_t sizes[] = {2, 3, 17, 257, 512, 1000, 1024, 2048, 2049, 3000, 4096, 5000, 8192, 12288};
  int plans = 0;
  for (int t = 0; t < 400; ++t) {
    const int32_t np = 1 + static_cast<int32_t>(g() % 64);
    std::vector<dtm_scene> sc(np);
    for (auto& s : sc) s = make(g, sizes[g() % (sizeof(sizes) / sizeof(sizes[0]))]);
    if (t % 50 == 0) sc[0].n_bins = 65536;
    const dtm_dtype dt = (t & 1) ? DTM_F32 : DTM_F64;
    // each field valid most of the time; the plan must be refused exactly
    // when one is not
    const bool spoil = g() % 4 == 0;
    const int which = static_cast<int>(g() % 8);
    dtm_tile_config tc{};
    const int32_t rows[] = {0, 16, 48, 64, 1024, 8192};
    tc.band_rows = rows[g() % 6];
    const int32_t cpts[] = {0, 1, 2, 4};
    tc.band_cpt = cpts[g() % 4];
    tc.fused_max_bins = g() % 3 == 0 ? 0 : 2 + static_cast<int32_t>(g() % 5000);
    tc.fused_threads = g() % 3 == 0 ? 512 : g() % 2 ? 256 : 0;
    const int32_t unrolls[] = {0, 2, 4, 8};
    tc.fused_unroll = unrolls[g() % 4];
    const int32_t max_iter = 1 + static_cast<int32_t>(g() % 100);
    tc.dense_sweeps = static_cast<int32_t>(g() % (max_iter + 1));
    tc.fused_blocks = static_cast<int32_t>(g() % 200);
    tc.band_min_items = static_cast<int32_t>(g() % 600);
    tc.independent_paths = static_cast<int32_t>(g() % 2);
    if (spoil) {
      switch (which) {
        case 0: tc.band_rows = g() % 2 ? 24 : 8208; break;
        case 1: tc.band_cpt = 3; break;
        case 2: tc.fused_threads = 128; break;
        case 3: tc.fused_unroll = 16; break;
        case 4: tc.dense_sweeps = max_iter + 1; break;
        case 5: tc.fused_blocks = -1; break;
        case 6: tc.band_min_items = -1; break;
        default: tc.independent_paths = 2; break;
      }
    }
    dtm_solve_opts o{1e-6, 0.25, max_iter, 4, DTM_STOP_BOUND, (g() % 2) ? DTM_FLAG_START_FLUX : 0};
    dtm_plan* p = nullptr;
    const int rc = dtm_plan_create(sc.data(), np, dt, &o, &tc, &p);
    EXPECT((rc == DTM_OK) == !spoil);
    if (rc != DTM_OK) {
      EXPECT(p == nullptr);
      continue;
    }
    ++plans;
    EXPECT(p != nullptr);
    EXPECT(dtm_plan_workspace_bytes(p) > 0);
    std::vector<int64_t> pi(np + 1), mat(np + 1);
    EXPECT(dtm_plan_offsets(p, pi.data(), mat.data()) == DTM_OK);
    int64_t acc = 0;
    for (int32_t q = 0; q < np; ++q) {
      EXPECT(pi[q] == acc);
      acc += sc[q].n_bins;
    }
    EXPECT(pi[np] == acc && dtm_plan_pi_elems(p) == acc);
    dtm_tile_config out{};
    EXPECT(dtm_plan_tiles(p, &out) == DTM_OK);
    EXPECT(out.band_rows >= 16 && out.band_rows % 16 == 0 && out.band_rows <= 8192);
    EXPECT(out.band_cpt == 1 || out.band_cpt == 2 || out.band_cpt == 4);
    EXPECT(out.dense_sweeps >= 1 && out.dense_sweeps <= o.max_iter && out.band_min_items >= 0);
    // every banded work item lies inside its pixel
    for (const dtm::BandItem& it : p->items) {
      const dtm::PixelMeta& m = p->meta[it.meta];
      EXPECT(it.band >= 0 && it.band < m.bands && static_cast<int64_t>(it.band) * out.band_rows < m.n);
      const int32_t colw = 256 * (dt == DTM_F32 ? 4 : 2) * out.band_cpt;
      EXPECT(it.colblock >= 0 && static_cast<int64_t>(it.colblock) * colw < m.n);
    }
    // the building sweep's finer items: only with column chunks, inside their pixel
    EXPECT(p->build_items.empty() == (out.band_cpt == 1 || p->items.empty()));
    for (const dtm::BandItem& it : p->build_items) {
      const dtm::PixelMeta& m = p->meta[it.meta];
      EXPECT(it.band >= 0 && it.band < m.bands && it.colblock >= 0 &&
             static_cast<int64_t>(it.colblock) * 256 * (dt == DTM_F32 ? 4 : 2) < m.n);
    }
    destroy(p);
  }
  // argument errors
  dtm_plan* p = reinterpret_cast<dtm_plan*>(0x1);
  dtm_scene one = make(g, 64);
  EXPECT(dtm_plan_create(nullptr, 1, DTM_F32, nullptr, nullptr, &p) == DTM_EINVAL && p == nullptr);
  EXPECT(dtm_plan_create(&one, 0, DTM_F32, nullptr, nullptr, &p) == DTM_EINVAL);
  EXPECT(dtm_plan_create(&one, 1, static_cast<dtm_dtype>(7), nullptr, nullptr, &p) == DTM_EINVAL);
  EXPECT(dtm_plan_create(&one, 1, DTM_F32, nullptr, nullptr, nullptr) == DTM_EINVAL);
  EXPECT(dtm_plan_offsets(nullptr, nullptr, nullptr) == DTM_EINVAL);
  EXPECT(dtm_plan_workspace_bytes(nullptr) == 0 && dtm_plan_pi_elems(nullptr) == -1);
  EXPECT(plans > 200);
  std::printf("host checks: %d plans made, %d failures\n", plans, failures);
  return failures == 0 ? 0 : 1;
}
