// Host-side argument checks of the library's C ABI under AddressSanitizer
// and UndefinedBehaviorSanitizer: brls_open's refusals (missing pointers,
// dimensions, sizes past the kernels' index ranges, bad velocities, the CFL
// bound), the entry points' refusals of NULL contexts and pointers, and a
// valid open (BRLS_EDEVICE without a GPU; on a GPU a context that opens,
// takes a shot, refuses bad ones, and closes). Test infrastructure: built
// and run by tests/test_sanitizers.py. Exit status 0 when every call
// returned what it should.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "brrlsm.h"

static int failures = 0;
#define EXPECT(cond, what)                    \
  do {                                        \
    if (!(cond)) {                            \
      std::fprintf(stderr, "FAILED: %s\n", what); \
      ++failures;                             \
    }                                         \
  } while (0)

static brls_grid grid64() {
  brls_grid g;
  std::memset(&g, 0, sizeof g);
  g.ndim = 2;
  g.nz = 64;
  g.ny = 1;
  g.nx = 64;
  g.nb = 20;
  g.nt_max = 500;
  g.nrec_max = 64;
  g.q_max = 2;
  g.h = 10.0;
  g.dt = 1e-3;
  g.lambda = 0.0;
  return g;
}

int main() {
  std::vector<float> vel(64 * 64, 2000.f);
  brls_ctx* c = nullptr;
  brls_grid g = grid64();
  EXPECT(brls_open(nullptr, vel.data(), nullptr, &c) == BRLS_EINVAL,
         "NULL grid");
  EXPECT(brls_open(&g, nullptr, nullptr, &c) == BRLS_EINVAL, "NULL velocity");
  EXPECT(brls_open(&g, vel.data(), nullptr, nullptr) == BRLS_EINVAL,
         "NULL out");
  EXPECT(std::strlen(brls_last_error(nullptr)) > 0, "message of a refusal");
  g.ndim = 4;
  EXPECT(brls_open(&g, vel.data(), nullptr, &c) == BRLS_EINVAL, "ndim 4");
  g = grid64();
  g.nb = 0;
  EXPECT(brls_open(&g, vel.data(), nullptr, &c) == BRLS_EINVAL, "nb 0");
  g = grid64();
  g.nt_max = 1;
  EXPECT(brls_open(&g, vel.data(), nullptr, &c) == BRLS_EINVAL, "nt_max 1");
  g = grid64();
  g.dt = -1.0;
  EXPECT(brls_open(&g, vel.data(), nullptr, &c) == BRLS_EINVAL, "dt < 0");
  g = grid64();
  g.lambda = std::nan("");
  EXPECT(brls_open(&g, vel.data(), nullptr, &c) == BRLS_EINVAL, "NaN lambda");
  g = grid64();
  g.nz = 1 << 15;
  g.nx = 1 << 15;  // 2^30 model points: past the 32-bit offsets
  EXPECT(brls_open(&g, vel.data(), nullptr, &c) == BRLS_EINVAL,
         "grid past the index range");
  g = grid64();
  g.nt_max = 1 << 20;
  g.nrec_max = 1 << 11;  // 2^31 samples per shot
  EXPECT(brls_open(&g, vel.data(), nullptr, &c) == BRLS_EINVAL,
         "samples per shot past the index range");
  g = grid64();
  std::vector<float> bad = vel;
  bad[100] = -1.f;
  EXPECT(brls_open(&g, bad.data(), nullptr, &c) == BRLS_EINVAL,
         "negative velocity");
  bad[100] = std::nanf("");
  EXPECT(brls_open(&g, bad.data(), nullptr, &c) == BRLS_EINVAL,
         "NaN velocity");
  std::vector<float> fast(64 * 64, 6000.f);  // v dt / h = 0.6 > 0.5546
  EXPECT(brls_open(&g, fast.data(), nullptr, &c) == BRLS_EINVAL, "CFL");
  EXPECT(c == nullptr, "no context after refusals");

  // every entry point refuses a NULL context
  float f = 0.f;
  double dv = 0.0;
  int32_t iv = 0;
  int64_t lv = 0;
  EXPECT(brls_update(nullptr, nullptr) != BRLS_OK, "update NULL");
  EXPECT(brls_downdate(nullptr, 0) != BRLS_OK, "downdate NULL");
  EXPECT(brls_solve_window(nullptr, 1, 0.0, nullptr) != BRLS_OK,
         "solve NULL");
  EXPECT(brls_image(nullptr, &f) != BRLS_OK, "image NULL");
  EXPECT(brls_image64(nullptr, &dv) != BRLS_OK, "image64 NULL");
  EXPECT(brls_set_image(nullptr, &f) != BRLS_OK, "set_image NULL");
  EXPECT(brls_apply_born(nullptr, &f, &f) != BRLS_OK, "born NULL");
  EXPECT(brls_apply_adjoint(nullptr, &f, &f) != BRLS_OK, "adjoint NULL");
  EXPECT(brls_apply_adjoint_static(nullptr, &f, &f) != BRLS_OK,
         "adjoint_static NULL");
  EXPECT(brls_set_precision(nullptr, 64, 64) != BRLS_OK, "precision NULL");
  EXPECT(brls_window_data_size(nullptr, &lv) != BRLS_OK, "size NULL");
  EXPECT(brls_tile_count(&iv) == BRLS_OK && iv > 0, "tile count");
  EXPECT(brls_tile_info(iv, &iv, &iv, &iv, &iv) == BRLS_EINVAL,
         "tile info past the last variant");
  brls_close(nullptr);

  // a valid grid: BRLS_EDEVICE without a GPU, else a working context
  g = grid64();
  const int rc = brls_open(&g, vel.data(), nullptr, &c);
  EXPECT(rc == BRLS_OK || rc == BRLS_EDEVICE, "valid grid");
  if (rc == BRLS_OK) {
    std::vector<int32_t> rec;
    for (int x = 0; x < 64; ++x) rec.insert(rec.end(), {2, 0, x});
    brls_shot s;
    std::memset(&s, 0, sizeof s);
    s.id = 7;
    s.sz = 2;
    s.sx = 32;
    s.nt = 500;
    s.nrec = 64;
    s.f0 = 15.0;
    s.rec = rec.data();
    EXPECT(brls_update(c, &s) == BRLS_OK, "update");
    EXPECT(brls_update(c, &s) == BRLS_EDUP, "duplicate id");
    s.id = 8;
    s.sx = 64;
    EXPECT(brls_update(c, &s) == BRLS_EINVAL, "source outside");
    s.sx = 32;
    s.nt = 501;
    EXPECT(brls_update(c, &s) == BRLS_EINVAL, "nt past nt_max");
    EXPECT(brls_downdate(c, 99) == BRLS_ENOSHOT, "downdate unknown");
    EXPECT(brls_set_precision(c, 16, 64) == BRLS_EINVAL, "precision 16");
    EXPECT(brls_set_exec(c, 9) == BRLS_EINVAL, "exec mode 9");
    EXPECT(brls_set_zchunk(c, 8) == BRLS_EINVAL, "z chunk in 2-D");
    brls_close(c);
  }
  if (failures) return 1;
  std::printf("ABI checks passed (open: %s)\n",
              rc == BRLS_OK ? "device" : "no device");
  return 0;
}
