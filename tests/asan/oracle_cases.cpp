// Runs the oracle on small cases written by the test, from host code built
// with AddressSanitizer, and compares the final conservative variables with
// those of the regular oracle build.  Case file: int64 header [D, nc, nf,
// nv, nbc, K, nsteps, order], double header [Pr, R, Tref, muref, omega, cfl,
// dt, 0], then 17 arrays, each an int64 byte count and its bytes: vol, cen,
// face_cells, face_area, face_normal, face_centroid, face_shift, face_bc,
// face_bc_id, u, w, bc kind, bc rho, bc U, bc T, W0, expected W.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

struct oracle_ctx;
extern "C" {
oracle_ctx* oracle_create(int D, int64_t nc, int64_t nf, const double* vol, const double* cen,
                          const int64_t* fcells, const double* farea, const double* fnorm,
                          const double* fcen, const double* fshift, const int32_t* fbc,
                          const int32_t* fbcid, int64_t nv, const double* u, const double* w,
                          int K, double Pr, double Rg, double Tref, double muref, double omega,
                          double cfl, double dt, int nbc, const int32_t* bckind, const double* bcrho,
                          const double* bcU, const double* bcT, const double* W0);
void oracle_set_order(oracle_ctx* o, int order);
int oracle_step(oracle_ctx* o, int nsteps, double* residual_out);
void oracle_get_state(const oracle_ctx* o, double* W, double* h, double* b, double* q);
const char* oracle_last_error(const oracle_ctx* o);
void oracle_destroy(oracle_ctx* o);
}

static int run(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) { std::printf("%s: cannot open\n", path); return 1; }
  int64_t hi[8];
  double hd[8];
  bool ok = std::fread(hi, sizeof hi, 1, f) == 1 && std::fread(hd, sizeof hd, 1, f) == 1;
  std::vector<std::vector<char>> a(17);
  for (auto& v : a) {
    int64_t n = 0;
    ok = ok && std::fread(&n, sizeof n, 1, f) == 1 && n >= 0;
    if (!ok) break;
    v.resize((size_t)n);
    ok = ok && (n == 0 || std::fread(v.data(), (size_t)n, 1, f) == 1);
  }
  std::fclose(f);
  if (!ok) { std::printf("%s: truncated\n", path); return 1; }
  auto d = [&](int i) { return a[i].empty() ? nullptr : (const double*)a[i].data(); };
  const int D = (int)hi[0];
  const int64_t nc = hi[1], nf = hi[2], nv = hi[3];
  oracle_ctx* o = oracle_create(D, nc, nf, d(0), d(1), (const int64_t*)a[2].data(), d(3), d(4), d(5),
                                d(6), (const int32_t*)a[7].data(), (const int32_t*)a[8].data(), nv,
                                d(9), d(10), (int)hi[5], hd[0], hd[1], hd[2], hd[3], hd[4], hd[5],
                                hd[6], (int)hi[4], (const int32_t*)a[11].data(), d(12), d(13), d(14),
                                d(15));
  if (!o) { std::printf("%s: oracle_create rejected the case\n", path); return 1; }
  if (hi[7] == 1) oracle_set_order(o, 1);
  double res[2];
  const int rc = oracle_step(o, (int)hi[6], res);
  if (rc) {
    std::printf("%s: oracle_step failed: %s\n", path, oracle_last_error(o));
    oracle_destroy(o);
    return 1;
  }
  std::vector<double> W((size_t)nc * (D + 2));
  oracle_get_state(o, W.data(), nullptr, nullptr, nullptr);
  oracle_destroy(o);
  const double* E = d(16);
  double err = 0.0, scale = 0.0;
  for (size_t i = 0; i < W.size(); ++i) {
    err = std::fmax(err, std::fabs(W[i] - E[i]));
    scale = std::fmax(scale, std::fabs(E[i]));
  }
  const bool same = err <= 1e-12 * scale;
  std::printf("%s: %lld steps, max |W - W_regular| / max|W| = %.3e%s\n", path, (long long)hi[6],
              err / scale, same ? "" : "  <-- differs");
  return same ? 0 : 1;
}

int main(int argc, char** argv) {
  int bad = 0;
  for (int i = 1; i < argc; ++i) bad += run(argv[i]);
  std::printf("%d cases, %d failed\n", argc - 1, bad);
  return bad ? 1 : 0;
}
