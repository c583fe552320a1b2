// Exercises the C-ABI entry points that run on the host alone (tile maps,
// argument checks, version, footprint) in a build whose host code carries
// AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status 0 = every
// check held and no sanitizer report ended the run.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/mpcr.h"

static int failures = 0;
#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                   \
    }                                                               \
  } while (0)

int main() {
  EXPECT(std::strlen(mpcr_version()) > 0);
  EXPECT(mpcr_last_error(nullptr) != nullptr);
  std::mt19937_64 g(7);
  for (int trial = 0; trial < 200; ++trial) {
    const int64_t nb = 128 * (1 + (int64_t)(g() % 4));
    const int64_t n = 1 + (int64_t)(g() % 5000);
    const int64_t nt = (n + nb - 1) / nb;
    const int nbands = 1 + (int)(g() % 4);
    std::vector<int> dmax(nbands), precs(nbands);
    int d = (int)(g() % 3);
    for (int b = 0; b < nbands; ++b) {
      dmax[b] = (b == nbands - 1) ? -1 : d;
      d += 1 + (int)(g() % 4);
      precs[b] = b == 0 ? MPCR_FP64 : (int)(g() % 5);
    }
    std::vector<uint8_t> band((size_t)(nt * nt), 0xAB), out((size_t)(nt * nt), 0xCD);
    int rc = mpcr_tilemap_banded(n, nb, dmax.data(), precs.data(), nbands, band.data());
    EXPECT(rc == MPCR_OK);
    if (rc != MPCR_OK) continue;
    for (int64_t i = 0; i < nt; ++i) {
      EXPECT(band[(size_t)(i * nt + i)] == MPCR_FP64);
      for (int64_t j = 0; j <= i; ++j) EXPECT(band[(size_t)(i * nt + j)] <= MPCR_FP8_E4M3);
    }
    std::vector<double> amax((size_t)(nt * nt), 0.0);
    for (auto& a : amax) a = std::exp(-20.0 * (double)(g() % 1000) / 1000.0);
    const double guard = std::ldexp(1.0, -(int)(g() % 30));
    rc = mpcr_tilemap_guarded(n, nb, band.data(), amax.data(), guard, out.data());
    EXPECT(rc == MPCR_OK);
    for (int64_t i = 0; i < nt && rc == MPCR_OK; ++i)
      for (int64_t j = 0; j <= i; ++j) {
        const int p = out[(size_t)(i * nt + j)], q = band[(size_t)(i * nt + j)];
        EXPECT(p <= MPCR_FP8_E4M3);
        EXPECT(!(q == MPCR_FP64 && p != MPCR_FP64));  // the guard only promotes
      }
    EXPECT(mpcr_serve_footprint(n, nb) > 0);
  }
  // argument checks
  std::vector<uint8_t> m(16);
  int dm[1] = {-1}, pr[1] = {MPCR_FP64};
  EXPECT(mpcr_tilemap_banded(-1, 128, dm, pr, 1, m.data()) != MPCR_OK);
  EXPECT(mpcr_tilemap_banded(1000, 128, nullptr, pr, 1, m.data()) != MPCR_OK);
  int bad[1] = {7};
  EXPECT(mpcr_tilemap_banded(256, 128, dm, bad, 1, m.data()) != MPCR_OK);   // unknown format
  EXPECT(mpcr_tilemap_guarded(256, 128, nullptr, nullptr, 1.0, m.data()) != MPCR_OK);
  EXPECT(mpcr_ctx_destroy(nullptr) != MPCR_OK);
  if (failures) std::fprintf(stderr, "%d check(s) failed\n", failures);
  return failures ? 1 : 0;
}
