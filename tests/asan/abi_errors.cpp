// Drives the library's argument checks and error returns from host code.
// Built with AddressSanitizer on the host side of every library source, it
// runs without a GPU: each invalid call must return its status before any
// device call, and a valid call must fail cleanly at the first device call
// (no device present), releasing what it had allocated.
#include <cstdio>
#include <cstring>
#include "ugks.h"

static int checks = 0, bad = 0;

// msg == nullptr: the call sets no message (the tuning-file calls)
static void expect(const char* what, int got, int want, const char* msg) {
  ++checks;
  const bool ok = got == want && (msg == nullptr || msg[0] != '\0');
  std::printf("%-26s %4d  %s%s\n", what, got, msg ? msg : "-", ok ? "" : "  <-- unexpected");
  if (!ok) ++bad;
}

int main() {
  // one unit square cell, four walls
  double vol[1] = {1.0}, cen[2] = {0.5, 0.5};
  int64_t fc[8] = {0, -1, 0, -1, 0, -1, 0, -1};
  double area[4] = {1, 1, 1, 1};
  double nrm[8] = {0, -1, 1, 0, 0, 1, -1, 0};
  double fcen[8] = {0.5, 0, 1, 0.5, 0.5, 1, 0, 0.5};
  int32_t fbc[4] = {1, 1, 1, 1}, fid[4] = {0, 0, 0, 0};
  ugks_mesh m{};
  m.dim = 2; m.n_cells = 1; m.n_faces = 4; m.cell_volume = vol; m.cell_centroid = cen;
  m.face_cells = fc; m.face_area = area; m.face_normal = nrm; m.face_centroid = fcen;
  m.face_shift = nullptr; m.face_bc = fbc; m.face_bc_id = fid;
  double u[8] = {-0.5, -0.5, -0.5, 0.5, 0.5, -0.5, 0.5, 0.5}, w[4] = {1, 1, 1, 1};
  ugks_velocity v{}; v.nv = 4; v.u = u; v.w = w;
  ugks_gas g{}; g.K = 0; g.Pr = 2.0 / 3.0; g.R = 0.5; g.T_ref = 1; g.mu_ref = 0.05; g.omega = 0.5; g.cfl = 0.8;
  ugks_bc bc{}; bc.kind = 1; bc.rho = 1; bc.T = 1;
  double W0[4] = {1, 0, 0, 0.75};
  ugks_ctx* c = nullptr;
  auto create = [&]() { return ugks_create(&m, &v, &g, &bc, 1, W0, nullptr, &c); };
  auto err = []() { return ugks_last_error(nullptr); };

  expect("out is NULL", ugks_create(&m, &v, &g, &bc, 1, W0, nullptr, nullptr), UGKS_EINVAL, err());
  expect("mesh is NULL", ugks_create(nullptr, &v, &g, &bc, 1, W0, nullptr, &c), UGKS_EINVAL, err());
  vol[0] = -1; expect("negative volume", create(), UGKS_EINVAL, err()); vol[0] = 1;
  nrm[0] = 2; expect("non-unit normal", create(), UGKS_EINVAL, err()); nrm[0] = 0;
  w[0] = 0; expect("zero weight", create(), UGKS_EINVAL, err()); w[0] = 1;
  fid[2] = 7; expect("bc id out of range", create(), UGKS_EINVAL, err()); fid[2] = 0;
  W0[0] = 0; expect("zero density", create(), UGKS_EINVAL, err()); W0[0] = 1;
  area[1] = 1.5; expect("cell not closed", create(), UGKS_EINVAL, err()); area[1] = 1;
  fc[2] = 5; expect("cell index out of range", create(), UGKS_EINVAL, err()); fc[2] = 0;
  g.K = -1; expect("negative internal dof", create(), UGKS_EINVAL, err()); g.K = 0;
  m.n_cells = 0; expect("empty mesh", create(), UGKS_EINVAL, err()); m.n_cells = 1;
  v.nv = 0; expect("empty velocity set", create(), UGKS_EINVAL, err()); v.nv = 4;
  // valid: stops at the first device call, nothing leaks
  c = nullptr;
  const int rc = create();
  ++checks;
  std::printf("%-26s %4d  %s\n", "valid, no device", rc, err());
  if (rc == UGKS_OK) ugks_destroy(c);
  else if (rc != UGKS_EHIP || c != nullptr) ++bad;

  expect("step on NULL", ugks_step(nullptr, 1, nullptr), UGKS_EINVAL, err());
  expect("moments on NULL", ugks_moments(nullptr, 0, nullptr, 0), UGKS_EINVAL, err());
  ugks_batch* b = nullptr;
  expect("batch of none", ugks_batch_create(nullptr, 0, nullptr, &b), UGKS_EINVAL,
         ugks_batch_last_error(nullptr));
  // the batch checks its options before any device call
  ugks_case cs[2] = {{&m, &v, &g, &bc, 1, W0}, {&m, &v, &g, &bc, 1, W0}};
  ugks_options o{};
  o.precision = 7;
  expect("batch, bad precision", ugks_batch_create(cs, 2, &o, &b), UGKS_EINVAL,
         ugks_batch_last_error(nullptr));
  o.precision = 0;
  o.block_v = 100;
  expect("batch, bad block_v", ugks_batch_create(cs, 2, &o, &b), UGKS_EINVAL,
         ugks_batch_last_error(nullptr));
  // each case's arguments are checked before any device call too
  cs[1].mesh = nullptr;
  expect("batch, case without mesh", ugks_batch_create(cs, 2, nullptr, &b), UGKS_EINVAL,
         ugks_batch_last_error(nullptr));
  cs[1].mesh = &m;
  ugks_gas g2 = g;
  g2.K = 2;
  cs[1].gas = &g2;
  expect("batch, case with K > 0", ugks_batch_create(cs, 2, nullptr, &b), UGKS_EUNSUPPORTED,
         ugks_batch_last_error(nullptr));
  cs[1].gas = &g;
  ugks_mesh m3 = m;
  m3.dim = 3;
  cs[1].mesh = &m3;
  expect("batch, mixed dimension", ugks_batch_create(cs, 2, nullptr, &b), UGKS_EINVAL,
         ugks_batch_last_error(nullptr));
  cs[1].mesh = &m;
  ugks_mlp* net = nullptr;
  expect("mlp params NULL", ugks_mlp_create(nullptr, nullptr, nullptr, nullptr, &net), UGKS_EINVAL,
         ugks_mlp_last_error(nullptr));
  expect("tuning file missing", ugks_autotune_load("/nonexistent/ugks_tune.txt"), UGKS_EINVAL, nullptr);
  expect("tuning path NULL", ugks_autotune_save(nullptr), UGKS_EINVAL, nullptr);
  ugks_destroy(nullptr);
  ugks_batch_destroy(nullptr);
  ugks_mlp_destroy(nullptr);
  std::printf("%d checks, %d unexpected\n", checks, bad);
  return bad ? 1 : 0;
}
