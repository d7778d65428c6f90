// Host-side check of the C ABI's argument validation under AddressSanitizer
// and UndefinedBehaviorSanitizer (host code only; no GPU is touched): every
// call below must be refused before any device work, with a status and a
// message, and nothing may read or write out of bounds on the way.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "slim.h"
#include "slim3d.h"
#include "slim_cnn.h"

static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

static void expect_einval(slim_status s, const char* what) {
  expect(s == SLIM_EINVAL, what);
  expect(std::strlen(slim_last_error()) > 0, what);
}

int main() {
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const double inf = std::numeric_limits<double>::infinity();
  slim_opts o;
  expect(slim_default_opts(&o) == SLIM_OK, "default opts");
  expect(slim_default_opts(nullptr) == SLIM_EINVAL, "default opts NULL");
  for (int s = -1; s <= 8; ++s) expect(slim_strerror((slim_status)s) != nullptr, "strerror");

  // slim_init: every argument outside its range
  slim_ctx* c = nullptr;
  slim_grid g{64, 1};
  double angles[90];
  for (int a = 0; a < 90; ++a) angles[a] = a * 3.14159265358979 / 90;
  expect_einval(slim_init(nullptr, &g, 90, nullptr, 91, 5, 1e-2, &o), "init out NULL");
  expect_einval(slim_init(&c, nullptr, 90, nullptr, 91, 5, 1e-2, &o), "init grid NULL");
  const int bad_n[] = {-5, 0, 1, 8193};
  for (int n : bad_n) {
    slim_grid gb{n, 1};
    expect_einval(slim_init(&c, &gb, 90, nullptr, 91, 5, 1e-2, &o), "init N");
  }
  slim_grid g0{64, 0};
  expect_einval(slim_init(&c, &g0, 90, nullptr, 91, 5, 1e-2, &o), "init n_slices");
  expect_einval(slim_init(&c, &g, 0, nullptr, 91, 5, 1e-2, &o), "init n_angles");
  expect_einval(slim_init(&c, &g, 90, nullptr, 0, 5, 1e-2, &o), "init n_rays 0");
  expect_einval(slim_init(&c, &g, 90, nullptr, 4097, 5, 1e-2, &o), "init n_rays big");
  expect_einval(slim_init(&c, &g, 90, nullptr, 91, -1, 1e-2, &o), "init r");
  const double bad_lam[] = {0.0, -1.0, nan, inf};
  for (double l : bad_lam) expect_einval(slim_init(&c, &g, 90, nullptr, 91, 5, l, &o), "init lambda");
  angles[17] = nan;
  expect_einval(slim_init(&c, &g, 90, angles, 91, 5, 1e-2, &o), "init NaN angle");
  angles[17] = 0.5;
  slim_opts ob = o;
  ob.angles_per_block = 7;
  expect_einval(slim_init(&c, &g, 90, nullptr, 91, 5, 1e-2, &ob), "init g");
  ob = o;
  ob.angles_per_block = 2;
  expect_einval(slim_init(&c, &g, 90, nullptr, 91, 200, 1e-2, &ob), "init window list");
  ob = o;
  ob.precision = 7;
  expect_einval(slim_init(&c, &g, 90, nullptr, 91, 5, 1e-2, &ob), "init precision");
  ob = o;
  ob.gram_mode = 9;
  expect_einval(slim_init(&c, &g, 90, nullptr, 91, 5, 1e-2, &ob), "init gram mode");
  ob = o;
  ob.gram_mode = SLIM_GRAM_CHOL;
  ob.angles_per_block = 4;
  slim_grid g5{512, 1};
  expect_einval(slim_init(&c, &g5, 360, nullptr, 725, 8, 1e-3, &ob), "init explicit Gram too big");
  ob = o;
  ob.check_every = 0;
  expect_einval(slim_init(&c, &g, 90, nullptr, 91, 5, 1e-2, &ob), "init check_every");
  ob = o;
  ob.damping_ramp = 2;
  expect_einval(slim_init(&c, &g, 90, nullptr, 91, 5, 1e-2, &ob), "init ramp");
  ob = o;
  ob.tikhonov = nan;
  expect_einval(slim_init(&c, &g, 90, nullptr, 91, 5, 1e-2, &ob), "init tikhonov");
  ob = o;
  ob.tikhonov = 0.1;
  ob.precision = SLIM_PREC_BF16;
  expect_einval(slim_init(&c, &g, 90, nullptr, 91, 5, 1e-2, &ob), "init tikhonov bf16");
  ob = o;
  ob.pcg_max_iter = 0;
  expect_einval(slim_init(&c, &g, 90, nullptr, 91, 5, 1e-2, &ob), "init pcg");
  expect(c == nullptr, "no context after refusals");

  // every entry point refuses a NULL context or group
  int32_t ids[2] = {0, 1};
  double norms[3];
  int64_t sz = 0;
  double ms = 0;
  int64_t nl = 0;
  slim_step_info info;
  slim_solve_info sinfo;
  slim_tune t{};
  slim_tune_info ti;
  expect_einval(slim_set_data(nullptr, nullptr, nullptr, nullptr), "set_data");
  expect_einval(slim_step(nullptr, ids, 2, &info), "step");
  expect_einval(slim_step_data(nullptr, ids, 2, nullptr, &info), "step_data");
  expect_einval(slim_set_lambda(nullptr, 1.0), "set_lambda");
  expect_einval(slim_slice_norms(nullptr, norms, 1), "slice_norms");
  expect_einval(slim_solve(nullptr, nullptr, nullptr, nullptr, 1e-2, 1, &sinfo), "solve");
  expect_einval(slim_project(nullptr, ids, 2, nullptr, nullptr), "project");
  expect_einval(slim_project_noalloc(nullptr, ids, 2, nullptr, nullptr), "project_noalloc");
  expect_einval(slim_backproject(nullptr, ids, 2, nullptr, nullptr), "backproject");
  expect_einval(slim_data_backprojection(nullptr, ids, 2, nullptr), "data_backprojection");
  expect_einval(slim_gram(nullptr, ids, 1, ids, 1, nullptr), "gram");
  expect_einval(slim_get_state(nullptr, nullptr, &sz), "get_state");
  expect_einval(slim_set_state(nullptr, nullptr, 0), "set_state");
  expect_einval(slim_autotune(nullptr, 0, 0, &ti), "autotune");
  expect_einval(slim_set_tune(nullptr, &t), "set_tune");
  expect_einval(slim_get_tune(nullptr, &t), "get_tune");
  expect_einval(slim_profile(nullptr, 1), "profile");
  expect_einval(slim_kernel_stats(nullptr, 0, &ms, &nl), "kernel_stats");
  expect_einval(slim_group_create(nullptr, nullptr, 0), "group_create");
  expect_einval(slim_group_step(nullptr, ids, 2, &info), "group_step");
  expect_einval(slim_group_set_shared(nullptr, 1), "group_set_shared");
  slim_group_destroy(nullptr);
  slim_destroy(nullptr);

  // the 3D context
  slim3d_ctx* c3 = nullptr;
  double dirs[4 * 3] = {0, 0, 1, 1, 0, 0, 0, 1, 0, 0.6, 0.8, 0};
  expect_einval(slim3d_init(nullptr, 16, 4, dirs, 16, 0, 1e-2, &o), "3d out");
  expect_einval(slim3d_init(&c3, 1, 4, dirs, 16, 0, 1e-2, &o), "3d N");
  expect_einval(slim3d_init(&c3, 2048, 4, dirs, 16, 0, 1e-2, &o), "3d N big");
  expect_einval(slim3d_init(&c3, 16, 0, dirs, 16, 0, 1e-2, &o), "3d n_dirs");
  expect_einval(slim3d_init(&c3, 16, 4, nullptr, 16, 0, 1e-2, &o), "3d dirs NULL");
  expect_einval(slim3d_init(&c3, 16, 4, dirs, 0, 0, 1e-2, &o), "3d n_det");
  expect_einval(slim3d_init(&c3, 16, 4, dirs, 16, -1, 1e-2, &o), "3d r");
  expect_einval(slim3d_init(&c3, 16, 4, dirs, 16, 0, nan, &o), "3d lambda");
  dirs[3] = 2.0;
  expect_einval(slim3d_init(&c3, 16, 4, dirs, 16, 0, 1e-2, &o), "3d unit length");
  dirs[3] = nan;
  expect_einval(slim3d_init(&c3, 16, 4, dirs, 16, 0, 1e-2, &o), "3d NaN direction");
  dirs[3] = 1.0;
  ob = o;
  ob.angles_per_block = 3;
  expect_einval(slim3d_init(&c3, 16, 4, dirs, 16, 0, 1e-2, &ob), "3d g");
  ob = o;
  ob.gram_mode = SLIM_GRAM_CHOL;
  expect_einval(slim3d_init(&c3, 16, 4, dirs, 16, 0, 1e-2, &ob), "3d chol");
  ob = o;
  ob.tikhonov = 0.5;
  expect_einval(slim3d_init(&c3, 16, 4, dirs, 16, 0, 1e-2, &ob), "3d tikhonov");
  expect(c3 == nullptr, "no 3D context after refusals");
  expect_einval(slim3d_set_data(nullptr, nullptr, nullptr, nullptr), "3d set_data");
  expect_einval(slim3d_step(nullptr, ids, 1, &info), "3d step");
  expect_einval(slim3d_project(nullptr, ids, 1, nullptr, nullptr), "3d project");
  expect_einval(slim3d_backproject(nullptr, ids, 1, nullptr, nullptr), "3d backproject");
  expect_einval(slim3d_kernel_stats(nullptr, 0, &ms, &nl), "3d kernel_stats");
  slim3d_destroy(nullptr);

  // the network
  slim_cnn* net = nullptr;
  slim_cnn_desc d{64, 2, {32, 64, 0, 0}, 1, 1.0, nullptr};
  slim_cnn_desc db = d;
  db.N = 60;
  expect_einval(slim_cnn_create(&net, &db), "cnn N");
  db = d;
  db.levels = 5;
  expect_einval(slim_cnn_create(&net, &db), "cnn levels");
  db = d;
  db.channels[1] = 48;
  expect_einval(slim_cnn_create(&net, &db), "cnn channels");
  db = d;
  db.max_batch = 0;
  expect_einval(slim_cnn_create(&net, &db), "cnn batch");
  db = d;
  db.in_scale = nan;
  expect_einval(slim_cnn_create(&net, &db), "cnn scale");
  expect_einval(slim_cnn_create(&net, nullptr), "cnn desc NULL");
  expect(slim_cnn_num_params(nullptr) == 0, "cnn params NULL");
  expect(slim_cnn_forward(nullptr, nullptr, nullptr, 1) == SLIM_EINVAL, "cnn forward NULL");
  slim_cnn_destroy(nullptr);

  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("validation: all checks passed\n");
  return 0;
}
