// Host-side paths of the C ABI, built with AddressSanitizer on the host code
// (tests/test_host_asan.py): argument validation, pyramid geometry, workspace
// layout and sizing, tunables, status strings and the profiling record.  Every
// call here returns before any device work, so no GPU is needed; a heap or
// stack overrun in the host code aborts the run with an ASan report.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lddmm.h"
#include "lddmm_cnn.h"
#include "lddmm_masks.h"

static int failures = 0;

#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) {                                                   \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                    \
    }                                                                \
  } while (0)

static lddmm_params params(int T, int levels) {
  lddmm_params p;
  std::memset(&p, 0, sizeof(p));
  p.alpha = 0.02;
  p.gamma = 1.0;
  p.sigma = 1.0;
  p.n_timesteps = T;
  p.n_levels = levels;
  for (int l = 0; l < LDDMM_MAX_LEVELS; ++l) p.iters[l] = 3;
  p.step = 0.02;
  p.guard = 1;
  p.weight[0] = 1.0;
  p.weight[1] = 0.5;
  return p;
}

static void sizes_and_grids() {
  const int dims[][3] = {{32, 32, 32}, {264, 160, 228}, {7, 9, 11}, {2, 2, 2}, {1024, 3, 2},
                         {97, 101, 103}};
  for (const auto& d : dims) {
    for (int L = 1; L <= 3; ++L) {
      for (int T : {1, 4, 10, LDDMM_MAX_T}) {
        lddmm_grid g{d[0], d[1], d[2], 0.05};
        lddmm_params p = params(T, L);
        const size_t ws = lddmm_workspace_size(&g, &p);
        int32_t P[3];
        int prev[3] = {0, 0, 0};
        for (int lev = L - 1; lev >= 0; --lev) {
          const int rc = lddmm_comp_grid(&g, &p, lev, P);
          if (rc != LDDMM_OK) continue;
          for (int a = 0; a < 3; ++a) {
            CHECK(P[a] >= 2 && P[a] <= LDDMM_MAX_DIM);
            if (prev[a]) CHECK(P[a] == 2 * prev[a]);   // the levels nest
            prev[a] = P[a];
          }
        }
        if (ws) {
          CHECK(lddmm_comp_grid(&g, &p, 0, P) == LDDMM_OK);
          CHECK(P[0] >= d[0] && P[1] >= d[1] && P[2] >= d[2]);
          // the workspace holds at least the two velocity buffers
          CHECK(ws >= 2ull * 3 * T * (size_t)P[0] * P[1] * P[2] * sizeof(float));
        }
        CHECK(lddmm_trace_rows(&p) == L * 4);
      }
    }
  }
  // invalid geometry or constants: size 0, EINVAL
  lddmm_grid g{32, 32, 32, 1.0};
  lddmm_params p = params(4, 1);
  lddmm_grid bad[] = {{1, 32, 32, 1.0}, {32, 0, 32, 1.0}, {32, 32, LDDMM_MAX_DIM + 1, 1.0},
                      {32, 32, 32, 0.0}, {32, 32, 32, -1.0}, {32, 32, 32, NAN},
                      {1024, 1024, 1024, 1.0}};
  for (auto& b : bad) {
    CHECK(lddmm_workspace_size(&b, &p) == 0);
    int32_t P[3];
    CHECK(lddmm_comp_grid(&b, &p, 0, P) == LDDMM_EINVAL);
  }
  lddmm_params q = p;
  q.n_timesteps = 0;
  CHECK(lddmm_workspace_size(&g, &q) == 0);
  q = p;
  q.n_timesteps = LDDMM_MAX_T + 1;
  CHECK(lddmm_workspace_size(&g, &q) == 0);
  q = p;
  q.sigma = 0.0;
  CHECK(lddmm_workspace_size(&g, &q) == 0);
  q = p;
  q.weight[0] = q.weight[1] = 0.0;
  CHECK(lddmm_workspace_size(&g, &q) == 0);
  q = p;
  q.n_levels = LDDMM_MAX_LEVELS + 1;
  int32_t P[3];
  CHECK(lddmm_comp_grid(&g, &q, 0, P) == LDDMM_EINVAL);
  CHECK(lddmm_comp_grid(&g, &p, 1, P) == LDDMM_EINVAL);     // one level only
  CHECK(lddmm_comp_grid(&g, &p, 0, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_trace_rows(nullptr) == 0);
  CHECK(lddmm_trace_rows(&q) == 0);
}

static void calls_rejected_before_launch() {
  lddmm_grid g{20, 24, 28, 0.1};
  lddmm_params p = params(4, 2);
  std::vector<float> host(16);
  float* fake = host.data();   // never dereferenced: every call below fails validation
  lddmm_problem pr;
  std::memset(&pr, 0, sizeof(pr));
  pr.grid = g;
  pr.template_mask = fake;
  pr.target_mask = fake;
  pr.v = fake;
  pr.workspace = fake;
  pr.workspace_bytes = 64;     // far too small
  CHECK(lddmm_register(&pr, 1, &p, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_register(&pr, 0, &p, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_register(nullptr, 1, &p, nullptr) == LDDMM_EINVAL);
  lddmm_problem two[2] = {pr, pr};
  int32_t st[2];
  CHECK(lddmm_register_batched(two, 2, &p, st, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_register_batched(two, 0, &p, st, nullptr) == LDDMM_EINVAL);
  double out4[4];
  CHECK(lddmm_energy(&pr, &p, out4, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_energy(&pr, &p, nullptr, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_gradient(&pr, &p, LDDMM_GRAD_V, fake, out4, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_gradient(&pr, &p, 7, fake, out4, nullptr) == LDDMM_EINVAL);
  lddmm_params rk = p;
  rk.flags = LDDMM_FLAG_RK4;
  pr.workspace_bytes = 1ull << 40;
  CHECK(lddmm_gradient(&pr, &rk, LDDMM_GRAD_L2, fake, out4, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_register_batched(two, 2, &rk, st, nullptr) == LDDMM_EINVAL);
  lddmm_problem noimg = pr;
  noimg.template_image = fake;   // image without a target image
  CHECK(lddmm_register(&noimg, 1, &p, nullptr) == LDDMM_EINVAL);
  // a problem beyond the static scratch is refused before anything runs
  lddmm_problem big = pr;
  big.grid = lddmm_grid{96, 96, 96, 1.0};
  lddmm_params p10 = params(10, 1);
  CHECK(lddmm_gradient_noalloc(&big, &p10, LDDMM_GRAD_V, fake, out4, nullptr) == LDDMM_ESCRATCH);
  CHECK(lddmm_gradient_noalloc(nullptr, &p10, LDDMM_GRAD_V, fake, out4, nullptr) == LDDMM_EINVAL);
  // apply, smooth and the helpers
  CHECK(lddmm_apply(&g, nullptr, fake, LDDMM_INTERP_LINEAR, LDDMM_F32, fake, nullptr) ==
        LDDMM_EINVAL);
  CHECK(lddmm_apply(&g, fake, fake, LDDMM_INTERP_LINEAR, LDDMM_I32, fake, nullptr) ==
        LDDMM_EINVAL);
  CHECK(lddmm_apply(&g, fake, fake, 5, LDDMM_F32, fake, nullptr) == LDDMM_EINVAL);
  const int32_t Pok[3] = {280, 160, 240}, Pbad[3] = {281, 160, 240};
  CHECK(lddmm_smooth_workspace_size(Pok) > 0);
  CHECK(lddmm_smooth_workspace_size(Pbad) == 0);
  CHECK(lddmm_smooth_workspace_size(nullptr) == 0);
  CHECK(lddmm_smooth(Pbad, 1.0, 0.02, 1.0, fake, fake, fake, 1ull << 40, nullptr) ==
        LDDMM_EINVAL);
  CHECK(lddmm_smooth(Pok, 1.0, 0.02, 1.0, fake, fake, fake, 16, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_make_mask(nullptr, fake, 0.1f, fake, fake, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_copy(nullptr, fake, 4, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_copy(fake, fake, -1, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_copy(nullptr, nullptr, 0, nullptr) == LDDMM_OK);
  // histogram matching, pre-alignment, masks
  lddmm_grid a{37, 41, 29, 1.0}, b{33, 35, 47, 1.0};
  CHECK(lddmm_histogram_match_workspace_size(&a, &b, 32) > 0);
  CHECK(lddmm_histogram_match_workspace_size(&a, &b, 0) == 0);
  CHECK(lddmm_histogram_match(&a, fake, fake, &b, fake, fake, 0, 8, fake, nullptr, nullptr, fake,
                              1ull << 30, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_histogram_match(&a, fake, fake, &b, fake, fake, 32, 8, fake, nullptr, nullptr,
                              fake, 8, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_align_workspace_size(&b) > 0);
  lddmm_align_params ap{LDDMM_ALIGN_RIGID, 10, 0.0, 10};
  double aff[12];
  CHECK(lddmm_align(&a, fake, &b, fake, &ap, aff, nullptr, fake, 1ull << 30, nullptr) ==
        LDDMM_EINVAL);
  CHECK(lddmm_masks_workspace_size(&a) > 0);
  CHECK(lddmm_morphology(&a, fake, 99, 2.0, fake, fake, 1ull << 30, nullptr) == LDDMM_EINVAL);
  CHECK(lddmm_morphology(&a, fake, 0, -1.0, fake, fake, 1ull << 30, nullptr) == LDDMM_EINVAL);
  // convolution helpers
  lddmm_cnn_shape xs{1, 8, 8, 8, 2};
  CHECK(lddmm_conv3d_wgrad_workspace(xs, 16, 1) > 0);
  CHECK(lddmm_cnn_mse_workspace(1000) > 0);
  CHECK(lddmm_cnn_expand_velocity(nullptr, 10, 24, 24, 24, 1.f, fake, fake, nullptr) ==
        LDDMM_EINVAL);
}

static void tunables_strings_profile() {
  for (int which = 0; which <= 6; ++which) {
    CHECK(lddmm_set_tunable(which, 0) == (which == LDDMM_TUNE_FWD_TILES ? LDDMM_OK : LDDMM_EINVAL));
    CHECK(lddmm_set_tunable(which, 1 << 30) == LDDMM_OK);
  }
  CHECK(lddmm_set_tunable(LDDMM_TUNE_FFT_FUSED_LDS, -1) == LDDMM_EINVAL);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_FFT_FUSED_LDS, 0) == LDDMM_OK);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_FFT_FUSED_LDS, 81920) == LDDMM_OK);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_K_TIME_BATCH, -1) == LDDMM_EINVAL);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_K_TIME_BATCH, 2) == LDDMM_EINVAL);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_K_TIME_BATCH, 0) == LDDMM_OK);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_K_TIME_BATCH, 1) == LDDMM_OK);
  CHECK(lddmm_set_tunable(99, 1) == LDDMM_EINVAL);
  CHECK(lddmm_set_tunable(-1, 1) == LDDMM_EINVAL);
  // back to the defaults
  CHECK(lddmm_set_tunable(LDDMM_TUNE_SWEEP_BLOCKS, 4096) == LDDMM_OK);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_FFT_X_ELEMS, 2048) == LDDMM_OK);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_FFT_COLS, 16) == LDDMM_OK);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_FFT_ZCOLS, 8) == LDDMM_OK);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_STAGED_MIN_BLOCKS, 2048) == LDDMM_OK);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_FWD_TILES, 1792) == LDDMM_OK);
  CHECK(lddmm_set_tunable(LDDMM_TUNE_FWD_STAGED_MIN_BLOCKS, 2048) == LDDMM_OK);
  for (int code = -10; code <= 10; ++code) {
    const char* s = lddmm_strerror(code);
    CHECK(s != nullptr && std::strlen(s) > 0);
  }
  CHECK(lddmm_profile_begin(0xFFFFFFFFu, 0) == LDDMM_OK);
  double ms[LDDMM_PROF_CLASSES];
  int64_t cnt[LDDMM_PROF_CLASSES], vox[LDDMM_PROF_CLASSES];
  CHECK(lddmm_profile_end(ms, cnt, vox) == LDDMM_OK);
  for (int k = 0; k < LDDMM_PROF_CLASSES; ++k) CHECK(cnt[k] == 0 && ms[k] == 0.0);
  CHECK(lddmm_profile_end(nullptr, nullptr, nullptr) == LDDMM_OK);
}

int main() {
  sizes_and_grids();
  calls_rejected_before_launch();
  tunables_strings_profile();
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host ABI checks passed\n");
  return 0;
}
