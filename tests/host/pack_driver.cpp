// Host-only driver of the table packer for sanitizer builds (AddressSanitizer
// and UndefinedBehaviorSanitizer): packs DIS and hadronic tables of edge
// shapes in every storage format and checks what the packer promises
// without decoding the fragment order: every scale is a power of two that
// bounds its row, the packed sizes cover the groups, and packing is
// deterministic.  Any out-of-bounds access or undefined behaviour aborts.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "pack.h"

using namespace fk;

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                     \
    }                                                              \
  } while (0)

static void check_scales(const PackedTable &pt, const std::vector<double> &rowmax, double qmax) {
  CHECK(pt.scale.size() == rowmax.size());
  for (size_t i = 0; i < rowmax.size(); ++i) {
    const double s = pt.scale[i];
    int e = 0;
    CHECK(std::frexp(s, &e) == 0.5);  // a power of two
    if (rowmax[i] > 0) {
      CHECK(rowmax[i] / s <= qmax);
      CHECK(rowmax[i] / (s / 2) > qmax);  // the smallest such power
    }
  }
}

int main() {
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd;
  const int dtypes[3] = {FK_F32, FK_BF16, FK_FP8E4M3};
  const double qmax[3] = {1.0, 1.0, 448.0};
  // DIS: (N, F, X, active flavours)
  const int dis_cases[][4] = {{1, 1, 2, 1}, {17, 14, 30, 9}, {33, 3, 128, 3}, {16, 64, 5, 40}};
  for (auto &cs : dis_cases) {
    const int N = cs[0], F = cs[1], X = cs[2], na = cs[3];
    std::vector<uint8_t> mask(F, 0);
    for (int a = 0; a < na; ++a) mask[(a * 7) % F] = 1;
    int nact = 0;
    for (int a = 0; a < F; ++a) nact += mask[a];
    std::vector<double> fk((size_t)N * nact * X);
    for (auto &v : fk) v = nd(rng);
    std::vector<double> rowmax(N, 0.0);
    for (int i = 0; i < N; ++i)
      for (size_t k = 0; k < (size_t)nact * X; ++k) rowmax[i] = std::max(rowmax[i], std::fabs(fk[i * (size_t)nact * X + k]));
    for (int d = 0; d < 3; ++d) {
      PackedTable p1, p2;
      pack_dis(fk.data(), mask.data(), N, F, X, dtypes[d], p1);
      pack_dis(fk.data(), mask.data(), N, F, X, dtypes[d], p2);
      CHECK(p1.fk == p2.fk && p1.fkT == p2.fkT);
      CHECK(p1.nact == nact);
      size_t units = 0;
      for (auto &g : p1.groups) units += (size_t)N * g.KE;
      CHECK(p1.fk.size() == units * 16);
      check_scales(p1, rowmax, qmax[d]);
    }
  }
  // hadronic: (N, F, X, pairs), general (non-symmetric) masks
  const int had_cases[][4] = {{1, 1, 2, 1}, {33, 14, 50, 60}, {5, 6, 7, 36}, {17, 64, 3, 100}};
  for (auto &cs : had_cases) {
    const int N = cs[0], F = cs[1], X = cs[2], np = cs[3];
    std::vector<uint8_t> mask((size_t)F * F, 0);
    int placed = 0;
    for (int k = 0; placed < np && k < F * F; ++k) {
      const int idx = (int)((k * 2654435761ull) % (unsigned)(F * F));
      if (!mask[idx]) {
        mask[idx] = 1;
        ++placed;
      }
    }
    std::vector<double> fk((size_t)N * placed * X * X);
    for (auto &v : fk) v = nd(rng);
    for (int d = 0; d < 3; ++d) {
      PackedTable p1, p2;
      pack_had(fk.data(), mask.data(), N, F, X, dtypes[d], p1);
      pack_had(fk.data(), mask.data(), N, F, X, dtypes[d], p2);
      CHECK(p1.fk == p2.fk && p1.fkT == p2.fkT);
      CHECK((int)p1.scale.size() == N);
      for (float s : p1.scale) {
        int e = 0;
        CHECK(std::frexp((double)s, &e) == 0.5);
      }
      CHECK(!p1.groups.empty() && !p1.agroups.empty());
    }
  }
  // rounding helpers at their edges
  CHECK(round_bf16(1.0) == 0x3f80);
  CHECK(round_bf16(-0.0) == 0x8000);
  CHECK(round_e4m3(448.0) == 0x7e);
  CHECK(round_e4m3(1e9) == 0x7e);      // saturating
  CHECK(round_e4m3(0.0009765625) == 0x00);  // 2^-10, half the smallest subnormal: ties to even
  CHECK(round_e4m3(0.0029296875) == 0x02);  // 1.5 * 2^-9: ties to even (2 * 2^-9)
  if (fails) {
    std::fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  std::printf("pack driver OK\n");
  return 0;
}
