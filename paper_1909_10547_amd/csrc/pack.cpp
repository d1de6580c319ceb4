// Host-side table packing: active-block compaction, the symmetric part of a
// hadronic table, per-datapoint power-of-two scales, rounding to the storage
// format and the fragment order the kernels stream.
#include "pack.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>

namespace fk {

// ---------------------------------------------------------------------------
// Rounding from binary64 (round to nearest, ties to even), done on the bit
// pattern of the double.
// ---------------------------------------------------------------------------
static inline uint64_t dbits(double x) {
  uint64_t b;
  std::memcpy(&b, &x, 8);
  return b;
}

// Shift right by s with round-to-nearest-even on the dropped bits.
static inline uint64_t shift_rne(uint64_t m, int s) {
  if (s <= 0) return m << (-s);
  if (s >= 64) return 0;
  const uint64_t keep = m >> s;
  const uint64_t rem = m & ((uint64_t(1) << s) - 1);
  const uint64_t half = uint64_t(1) << (s - 1);
  return keep + ((rem > half || (rem == half && (keep & 1))) ? 1 : 0);
}

uint16_t round_bf16(double x) {
  const uint64_t b = dbits(x);
  const uint16_t sign = (uint16_t)((b >> 48) & 0x8000);
  const int ex = (int)((b >> 52) & 0x7ff);
  const uint64_t frac = b & ((uint64_t(1) << 52) - 1);
  if (ex == 0x7ff) return frac ? 0x7fc0 : (uint16_t)(sign | 0x7f80);
  if (ex == 0) return sign;  // binary64 subnormals are far below bfloat16's range
  const int E = ex - 1023;
  const uint64_t mant = frac | (uint64_t(1) << 52);  // value = mant * 2^(E-52)
  if (E >= -126) {
    uint64_t keep = shift_rne(mant, 45);  // 8 significant bits
    int e = E;
    if (keep == 256) {
      keep = 128;
      ++e;
    }
    if (e > 127) return (uint16_t)(sign | 0x7f80);
    return (uint16_t)(sign | ((e + 127) << 7) | (keep & 0x7f));
  }
  // subnormal bfloat16: multiples of 2^-133
  const int s = -(E + 81);  // value / 2^-133 = mant * 2^(E - 52 + 133)
  return (uint16_t)(sign | (uint16_t)shift_rne(mant, s));
}

uint8_t round_e4m3(double x) {
  const uint64_t b = dbits(x);
  const uint8_t sign = (uint8_t)((b >> 56) & 0x80);
  const int ex = (int)((b >> 52) & 0x7ff);
  const uint64_t frac = b & ((uint64_t(1) << 52) - 1);
  if (ex == 0x7ff) return frac ? 0x7f : (uint8_t)(sign | 0x7e);  // NaN; inf saturates
  if (ex == 0) return sign;
  const int E = ex - 1023;
  const uint64_t mant = frac | (uint64_t(1) << 52);
  if (E >= -6) {
    uint64_t keep = shift_rne(mant, 49);  // 4 significant bits
    int e = E;
    if (keep == 16) {
      keep = 8;
      ++e;
    }
    if (e > 8 || (e == 8 && keep > 14)) return (uint8_t)(sign | 0x7e);  // saturate at 448
    return (uint8_t)(sign | ((e + 7) << 3) | (keep & 7));
  }
  const int s = 43 - E;  // value / 2^-9 = mant * 2^(E - 52 + 9)
  return (uint8_t)(sign | (uint8_t)shift_rne(mant, s));
}

double datapoint_scale(double absmax, double qmax) {
  if (!(absmax > 0.0) || !std::isfinite(absmax)) return 1.0;
  int e = (int)std::ceil(std::log2(absmax / qmax));
  while (absmax > qmax * std::ldexp(1.0, e)) ++e;
  while (absmax <= qmax * std::ldexp(1.0, e - 1)) --e;
  return std::ldexp(1.0, e);
}

static inline void store_elem(uint8_t *unit, int e, int dtype, double v) {
  if (dtype == FK_F32) {
    const float f = (float)v;
    std::memcpy(unit + 4 * e, &f, 4);
  } else if (dtype == FK_BF16) {
    const uint16_t h = round_bf16(v);
    std::memcpy(unit + 2 * e, &h, 2);
  } else {
    unit[e] = round_e4m3(v);
  }
}

static void parallel_for(int n, const std::function<void(int)> &fn) {
  int nt = (int)std::thread::hardware_concurrency();
  nt = std::max(1, std::min(nt, 32));
  if (n < 2 || nt == 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < std::min(nt, n); ++t)
    th.emplace_back([&]() {
      for (int i = next++; i < n; i = next++) fn(i);
    });
  for (auto &t : th) t.join();
}

// ---------------------------------------------------------------------------
// Splitting a concatenated contraction range into groups that fit in LDS
// ---------------------------------------------------------------------------
// ``blocks`` lists (source row of the block start, length) in k order.
static std::vector<GroupPlan> split_groups(int a, const std::vector<std::pair<int, int>> &blocks,
                                           int E, int nx) {
  std::vector<GroupPlan> out;
  long K = 0;
  for (auto &b : blocks) K += b.second;
  if (K == 0) return out;
  int kmax = kUnitsMax * E;
  kmax = std::min(kmax, ((kMaxSeg - 1) * nx) / E * E);
  kmax = std::max(kmax, E);
  const long ng = (K + kmax - 1) / kmax;
  long target = (K + ng - 1) / ng;
  target = (target + E - 1) / E * E;
  if (target > kmax) target = kmax;
  long k = 0;
  size_t bi = 0;
  int boff = 0;
  while (k < K) {
    GroupPlan g;
    g.a = a;
    long take = std::min(target, K - k);
    g.K = (int)take;
    while (take > 0) {
      const int len = (int)std::min<long>(blocks[bi].second - boff, take);
      g.seg_row.push_back(blocks[bi].first + boff);
      g.seg_len.push_back(len);
      take -= len;
      boff += len;
      if (boff == blocks[bi].second) {
        ++bi;
        boff = 0;
      }
    }
    g.KE = (g.K + E - 1) / E;
    k += g.K;
    out.push_back(g);
  }
  return out;
}

// ---------------------------------------------------------------------------
// DIS
// ---------------------------------------------------------------------------
void pack_dis(const double *fk, const uint8_t *mask, int N, int F, int X, int dtype,
              PackedTable &pt) {
  const int E = elems_per_unit(dtype);
  const double qmax = dtype == FK_FP8E4M3 ? 448.0 : 1.0;
  std::vector<int> flav;
  for (int a = 0; a < F; ++a)
    if (mask[a]) flav.push_back(a);
  const int nact = (int)flav.size();
  pt.nact = nact;
  pt.active = flav;
  // per-datapoint scale
  pt.scale.assign(N, 1.0f);
  parallel_for(N, [&](int i) {
    double m = 0;
    const double *row = fk + (size_t)i * nact * X;
    for (int k = 0; k < nact * X; ++k) m = std::max(m, std::fabs(row[k]));
    pt.scale[i] = (float)datapoint_scale(m, qmax);
  });
  // forward groups: k = (active flavour, x) concatenated
  std::vector<std::pair<int, int>> blocks;
  for (int a : flav) blocks.push_back({a * X, X});
  pt.groups = split_groups(-1, blocks, E, X);
  // each group's rows: datapoints; N*KE units
  size_t units = 0;
  for (auto &g : pt.groups) {
    g.base = units;
    units += (size_t)N * g.KE;
  }
  pt.fk.assign(units * 16, 0);
  // source column offset inside a datapoint row for a PDF row index
  std::vector<int> colof(F, -1);
  for (int c = 0; c < nact; ++c) colof[flav[c]] = c;
  const int nblk = (N + 15) / 16;
  for (auto &g : pt.groups) {
    std::vector<int> kcol(g.K);
    {
      int k = 0;
      for (size_t s = 0; s < g.seg_row.size(); ++s)
        for (int t = 0; t < g.seg_len[s]; ++t, ++k) {
          const int row = g.seg_row[s] + t;  // flavour*X + x
          kcol[k] = colof[row / X] * X + row % X;
        }
    }
    parallel_for(nblk, [&](int bl) {
      const int nv = std::min(16, N - 16 * bl);
      uint8_t *base = pt.fk.data() + (g.base + (size_t)bl * g.KE * 16) * 16;
      for (int u = 0; u < g.KE; ++u)
        for (int r = 0; r < nv; ++r) {
          const int i = 16 * bl + r;
          const double inv = 1.0 / pt.scale[i];
          uint8_t *unit = base + ((size_t)u * nv + r) * 16;
          for (int e = 0; e < E; ++e) {
            const int k = u * E + e;
            const double v = k < g.K ? fk[(size_t)i * nact * X + kcol[k]] * inv : 0.0;
            store_elem(unit, e, dtype, v);
          }
        }
    });
  }
  // transposed copy for the adjoint: rows (active flavour, x), k = datapoint
  const int nrows = nact * X;
  const int chunk = kDisChunkUnits * E;
  const int nch = (N + chunk - 1) / chunk;
  const int ntile = (nrows + 15) / 16;
  size_t tunits = 0;
  pt.tchunks.clear();
  for (int ch = 0; ch < nch; ++ch) {
    TChunk tc;
    tc.i0 = ch * chunk;
    tc.n = std::min(chunk, N - tc.i0);
    tc.KE = (tc.n + E - 1) / E;
    tc.base = tunits;
    tunits += (size_t)nrows * tc.KE;
    pt.tchunks.push_back(tc);
  }
  pt.fkT.assign(tunits * 16, 0);
  for (auto &tc : pt.tchunks) {
    parallel_for(ntile, [&](int tile) {
      const int nv = std::min(16, nrows - 16 * tile);
      uint8_t *base = pt.fkT.data() + (tc.base + (size_t)tile * 16 * tc.KE) * 16;
      for (int u = 0; u < tc.KE; ++u)
        for (int r = 0; r < nv; ++r) {
          const int row = 16 * tile + r;
          uint8_t *unit = base + ((size_t)u * nv + r) * 16;
          for (int e = 0; e < E; ++e) {
            const int k = u * E + e;
            double v = 0.0;
            if (k < tc.n) {
              const int i = tc.i0 + k;
              v = fk[(size_t)i * nact * X + row] / pt.scale[i];
            }
            store_elem(unit, e, dtype, v);
          }
        }
    });
  }
}

// ---------------------------------------------------------------------------
// hadronic
// ---------------------------------------------------------------------------
void pack_had(const double *fk, const uint8_t *mask, int N, int F, int X, int dtype,
              PackedTable &pt) {
  const int E = elems_per_unit(dtype);
  const double qmax = dtype == FK_FP8E4M3 ? 448.0 : 1.0;
  std::vector<int> pidx((size_t)F * F, -1);
  int np = 0;
  for (int a = 0; a < F; ++a)
    for (int b = 0; b < F; ++b)
      if (mask[a * F + b]) pidx[a * F + b] = np++;
  pt.npairs = np;
  const size_t blk = (size_t)X * X;
  auto in_sym = [&](int a, int b) { return pidx[a * F + b] >= 0 || pidx[b * F + a] >= 0; };
  // entry of the symmetric part S = FK + FK^T of datapoint i
  auto sval = [&](int i, int a, int b, int al, int be) -> double {
    double v = 0.0;
    const int p = pidx[a * F + b], q = pidx[b * F + a];
    if (p >= 0) v += fk[((size_t)i * np + p) * blk + (size_t)al * X + be];
    if (q >= 0) v += fk[((size_t)i * np + q) * blk + (size_t)be * X + al];
    return v;
  };
  // Row groups.  The forward sums Eq. (1) over unordered flavour pairs: row
  // flavour a takes the partners b >= a, with S_ab for b > a and S_aa / 2 on
  // the diagonal (an exact halving), so every product f_a f_b of the
  // bilinear form is stored once.  The adjoint needs S f over the whole
  // symmetric pattern, so it gets the full rows.
  auto row_groups = [&](bool upper) {
    std::vector<GroupPlan> out;
    for (int a = 0; a < F; ++a) {
      std::vector<std::pair<int, int>> blocks;
      for (int b = upper ? a : 0; b < F; ++b)
        if (in_sym(a, b)) blocks.push_back({b * X, X});
      auto g = split_groups(a, blocks, E, X);
      out.insert(out.end(), g.begin(), g.end());
    }
    return out;
  };
  pt.groups = row_groups(true);
  pt.agroups = row_groups(false);
  // per-datapoint scale from max |S_i| (shared by both copies)
  pt.scale.assign(N, 1.0f);
  parallel_for(N, [&](int i) {
    double m = 0;
    for (int a = 0; a < F; ++a)
      for (int b = a; b < F; ++b) {
        if (!in_sym(a, b)) continue;
        for (int al = 0; al < X; ++al)
          for (int be = 0; be < X; ++be) m = std::max(m, std::fabs(sval(i, a, b, al, be)));
      }
    pt.scale[i] = (float)datapoint_scale(m, qmax);
  });
  const int nblk = (N + 15) / 16;
  auto pack_groups = [&](std::vector<GroupPlan> &groups, std::vector<uint8_t> &buf, bool upper) {
    size_t units = 0;
    for (auto &g : groups) {
      g.base = units;
      units += (size_t)N * X * g.KE;
    }
    buf.assign(units * 16, 0);
    for (auto &g : groups) {
      std::vector<int> kb(g.K), kx(g.K);
      {
        int k = 0;
        for (size_t s = 0; s < g.seg_row.size(); ++s)
          for (int t = 0; t < g.seg_len[s]; ++t, ++k) {
            const int row = g.seg_row[s] + t;
            kb[k] = row / X;
            kx[k] = row % X;
          }
      }
      parallel_for(nblk, [&](int bl) {
        const int nv = std::min(16, N - 16 * bl);
        // Forward copy: the two blocks of a pair (2p, 2p+1) alternate at
        // every x index, [pair][alpha][block of the pair][unit][row], so the
        // waves that sweep alpha together read one contiguous window.  The
        // adjoint copy keeps [block][alpha][unit][row].
        const int b0 = upper ? bl & ~1 : bl;
        const int nv0 = std::min(16, N - 16 * b0);
        const int nv1 = upper && b0 + 1 < nblk ? std::min(16, N - 16 * (b0 + 1)) : 0;
        const size_t astride = upper ? (size_t)g.KE * (nv0 + nv1) : (size_t)g.KE * nv;
        const size_t toff = upper && bl != b0 ? (size_t)g.KE * nv0 : 0;
        uint8_t *bbase = buf.data() + (g.base + (size_t)b0 * X * g.KE * 16 + toff) * 16;
        for (int al = 0; al < X; ++al) {
          uint8_t *abase = bbase + al * astride * 16;
          for (int u = 0; u < g.KE; ++u)
            for (int r = 0; r < nv; ++r) {
              const int i = 16 * bl + r;
              const double inv = 1.0 / pt.scale[i];
              uint8_t *unit = abase + ((size_t)u * nv + r) * 16;
              for (int e = 0; e < E; ++e) {
                const int k = u * E + e;
                double v = 0.0;
                if (k < g.K) {
                  v = sval(i, g.a, kb[k], al, kx[k]) * inv;
                  if (upper && kb[k] == g.a) v *= 0.5;
                }
                store_elem(unit, e, dtype, v);
              }
            }
        }
      });
    }
  };
  pack_groups(pt.groups, pt.fk, true);
  pack_groups(pt.agroups, pt.fkT, false);
}

}  // namespace fk
