// Host runtime of the fkconv library: context, device-memory budget, table
// registry, launch plans and the non-serving C entry points.
#include "runtime.h"

#include <algorithm>
#include <map>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

using namespace fk;

namespace {
thread_local std::string g_create_err;

#define FK_TRY_HIP(c, expr)                                                            \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return set_err(c, FK_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct Guard {
  std::unique_lock<std::mutex> lk;
  explicit Guard(fk_ctx *c) : lk(c->mu) {}
};

}  // namespace

namespace fk {

fk_status set_err(fk_ctx *c, fk_status code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_create_err = buf;
  return code;
}

fk_status dev_alloc(fk_ctx *c, size_t bytes, void **p,
                    std::vector<std::pair<void *, size_t>> *track) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  uint64_t cur = c->used.load();
  for (;;) {
    if (cur + bytes > c->budget)
      return set_err(c, FK_E_BUDGET, "device-memory budget exhausted: %llu used + %llu requested > %llu",
                     (unsigned long long)cur, (unsigned long long)bytes,
                     (unsigned long long)c->budget);
    if (c->used.compare_exchange_weak(cur, cur + bytes)) break;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    c->used -= bytes;
    *p = nullptr;
    return set_err(c, FK_E_HIP, "hipMalloc(%llu): %s", (unsigned long long)bytes,
                   hipGetErrorString(e));
  }
  if (track) track->push_back({*p, bytes});
  return FK_OK;
}

void dev_free_all(fk_ctx *c, std::vector<std::pair<void *, size_t>> &track) {
  for (auto &a : track) {
    if (a.first) (void)hipFree(a.first);
    c->used -= a.second;
  }
  track.clear();
}

Plan *find_plan(fk_ctx *c, int64_t h) {
  auto it = c->plans.find(h);
  return it == c->plans.end() ? nullptr : it->second.get();
}
Table *find_table(fk_ctx *c, int64_t h) {
  auto it = c->tables.find(h);
  return it == c->tables.end() ? nullptr : it->second.get();
}

int pick_nt(int ncols) {
  const int t = (ncols + 15) / 16;
  if (t <= 1) return 1;
  if (t == 2) return 2;
  if (t <= 4) return 4;
  if (t <= 7) return 7;
  return 8;
}

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------
template <typename T>
static fk_status upload(fk_ctx *c, Plan &p, const std::vector<T> &v, T **dst) {
  void *d = nullptr;
  fk_status st = dev_alloc(c, std::max<size_t>(v.size(), 1) * sizeof(T), &d, &p.allocs);
  if (st) return st;
  if (!v.empty()) FK_TRY_HIP(c, hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *dst = (T *)d;
  return FK_OK;
}

// Lower the largest load of a static partition by local search: move an
// item of the most loaded list to a list where it ends below that load, or
// else swap it for a smaller item of another list, taking the exchange that
// leaves the smaller of the two new loads.  Which list runs an item does not
// change any result (each item writes its own partial slots).
static void rebalance(std::vector<std::vector<int>> &lists, std::vector<double> &load,
                      const std::vector<double> &cost) {
  const int G = (int)lists.size();
  for (int iter = 0; iter < 4 * G; ++iter) {
    const int mx = (int)(std::max_element(load.begin(), load.end()) - load.begin());
    const double M = load[mx];
    int best_j = -1, best_i = -1, best_k = -1;
    double best = M;
    for (int ii = 0; ii < (int)lists[mx].size(); ++ii) {
      const double ci = cost[lists[mx][ii]];
      for (int j = 0; j < G; ++j) {
        if (j == mx) continue;
        // move
        const double mv = std::max(M - ci, load[j] + ci);
        if (mv < best - 1e-9) {
          best = mv;
          best_j = j, best_i = ii, best_k = -1;
        }
        // swap with a smaller item of list j
        for (int kk = 0; kk < (int)lists[j].size(); ++kk) {
          const double ck = cost[lists[j][kk]];
          if (ck >= ci) continue;
          const double sw = std::max(M - ci + ck, load[j] + ci - ck);
          if (sw < best - 1e-9) {
            best = sw;
            best_j = j, best_i = ii, best_k = kk;
          }
        }
      }
    }
    if (best_j < 0) break;
    const int item = lists[mx][best_i];
    if (best_k < 0) {
      lists[mx].erase(lists[mx].begin() + best_i);
      lists[best_j].push_back(item);
      load[mx] -= cost[item];
      load[best_j] += cost[item];
    } else {
      const int other = lists[best_j][best_k];
      lists[mx][best_i] = other;
      lists[best_j][best_k] = item;
      load[mx] += cost[other] - cost[item];
      load[best_j] += cost[item] - cost[other];
    }
  }
  // longest items first in every list
  for (auto &l : lists)
    std::stable_sort(l.begin(), l.end(), [&](int x, int y) { return cost[x] > cost[y]; });
}

// Static work lists: items longest first to the least loaded of G lists,
// then the local search above.
static std::vector<std::vector<int>> partition_items(const std::vector<double> &cost, int G) {
  std::vector<int> order(cost.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<std::vector<int>> lists(G);
  std::vector<double> load(G, 0.0);
  std::vector<std::pair<double, int>> heap;  // (load, list), min-heap
  for (int g = 0; g < G; ++g) heap.push_back({0.0, g});
  auto cmp = [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
    return x.first != y.first ? x.first > y.first : x.second > y.second;
  };
  std::make_heap(heap.begin(), heap.end(), cmp);
  for (int k : order) {
    std::pop_heap(heap.begin(), heap.end(), cmp);
    lists[heap.back().second].push_back(k);
    heap.back().first += cost[k];
    load[heap.back().second] += cost[k];
    std::push_heap(heap.begin(), heap.end(), cmp);
  }
  rebalance(lists, load, cost);
  return lists;
}

static fk_status build_plan(fk_ctx *c, Plan &p, const std::vector<Table *> &ts) {
  const bool had = p.kind == FK_HAD;
  const int X = p.X, F = p.F;
  std::vector<GroupDesc> gd;
  std::vector<SegRef> segs;
  std::vector<std::vector<int>> segidx(ts.size());
  size_t bop = 0;
  // Descriptors that gather the same PDF rows (tables with the same flavour
  // pattern have the same groups) share one staged B operand, so a group
  // launch stages, and the forward kernels read, each distinct operand once.
  // Sharing stays within one phase (forward or adjoint), whose descriptors
  // the stage kernel walks as one contiguous range.
  std::map<std::vector<int>, int> same_b;
  std::vector<int32_t> rowtab;
  const int E = elems_per_unit(p.dtype);
  auto add_gd = [&](int a, int src, const std::vector<int> &rows, const std::vector<int> &lens,
                    int K, int KE) {
    std::vector<int> key;
    if (src == 0) {
      key = {a, K, KE, (int)rows.size()};
      key.insert(key.end(), rows.begin(), rows.end());
      key.insert(key.end(), lens.begin(), lens.end());
      auto it = same_b.find(key);
      if (it != same_b.end()) return it->second;
    }
    GroupDesc d;
    std::memset(&d, 0, sizeof d);
    // source row of every staged element, in k order: the segments
    // concatenated, -1 from K up to the whole k-step (KEpad units)
    d.row_off = (int64_t)rowtab.size();
    for (size_t q = 0; q < rows.size(); ++q)
      for (int e = 0; e < lens[q]; ++e) rowtab.push_back(rows[q] + e);
    rowtab.resize((size_t)d.row_off + (size_t)((KE + 3) / 4) * 4 * E, -1);
    d.a = a;
    d.src = src;
    d.nseg = (int)rows.size();
    d.K = K;
    d.KE = KE;
    d.bop_off = (int64_t)bop;
    for (size_t s = 0; s < rows.size(); ++s) {
      d.seg_row[s] = rows[s];
      d.seg_len[s] = lens[s];
    }
    bop += (size_t)((KE + 3) / 4) * 4 * kRpMax;
    gd.push_back(d);
    if (src == 0) same_b[key] = (int)gd.size() - 1;
    return (int)gd.size() - 1;
  };
  p.row0.clear();
  int row = 0;
  p.table_bytes = 0;
  for (auto *t : ts) {
    p.row0.push_back(row);
    row += t->N;
    p.table_bytes += t->fk_bytes + t->fkT_bytes;
  }
  p.Ntot = row;
  std::vector<float> scale_all;
  for (auto *t : ts) scale_all.insert(scale_all.end(), t->scale.begin(), t->scale.end());
  p.maxT_fwd = p.maxT_adj = 1;
  for (size_t t = 0; t < ts.size(); ++t)
    for (auto &g : ts[t]->groups) {
      const int gi = add_gd(g.a, 0, g.seg_row, g.seg_len, g.K, g.KE);
      segs.push_back({(const uint4 *)((const char *)ts[t]->d_fk + g.base * 16), gi, g.KE});
      segidx[t].push_back((int)segs.size() - 1);
      p.maxT_fwd = std::max(p.maxT_fwd, (g.KE + 3) / 4);
    }
  p.ngd_fwd = (int)gd.size();
  same_b.clear();
  std::vector<std::vector<int>> chunkgd(ts.size()), asegidx(ts.size());
  if (!had)
    for (size_t t = 0; t < ts.size(); ++t)
      for (auto &ch : ts[t]->tchunks) {
        chunkgd[t].push_back(add_gd(-1, 1, {p.row0[t] + ch.i0}, {ch.n}, ch.n, ch.KE));
        p.maxT_adj = std::max(p.maxT_adj, (ch.KE + 3) / 4);
      }
  else
    // the hadronic adjoint runs over the full symmetric rows (second copy)
    for (size_t t = 0; t < ts.size(); ++t)
      for (auto &g : ts[t]->agroups) {
        const int gi = add_gd(g.a, 0, g.seg_row, g.seg_len, g.K, g.KE);
        segs.push_back({(const uint4 *)((const char *)ts[t]->d_fkT + g.base * 16), gi, g.KE});
        asegidx[t].push_back((int)segs.size() - 1);
        p.maxT_adj = std::max(p.maxT_adj, (g.KE + 3) / 4);
      }
  p.ngd_adj = (int)gd.size() - p.ngd_fwd;

  // ---- forward items.  An item runs consecutive groups of one block (DIS:
  // of up to kWaves blocks) until about kItemUnits units per row are done.
  // The split depends on the table alone, so a table's result is bitwise
  // the same alone and inside any group.
  std::vector<FwdItem> items;
  std::vector<RedBlock> rblocks;
  std::vector<int32_t> slot_idx;
  const double target = kItemUnits;
  int nslots = 0;
  for (size_t t = 0; t < ts.size(); ++t) {
    const Table *T = ts[t];
    const int nblk = (T->N + 15) / 16;
    const int nG = (int)T->groups.size();
    std::vector<std::vector<int>> bslots(nblk);
    const int step = had ? 2 : kWaves;
    for (int b0 = 0; b0 < nblk; b0 += step) {
      const int nb = std::min(step, nblk - b0);
      int g = 0;
      while (g < nG) {
        const int g0 = g;
        double acc = 0;
        do {
          acc += (double)T->groups[g].KE * nb;
          ++g;
        } while (g < nG && acc + (double)T->groups[g].KE * nb <= target);
        FwdItem it;
        it.seg0 = segidx[t][g0];
        it.seg1 = segidx[t][g - 1] + 1;
        it.block0 = b0;
        it.nblk = nb;
        it.ndata = T->N;
        it.slot0 = nslots;
        for (int w = 0; w < nb; ++w) bslots[b0 + w].push_back(nslots + w);
        nslots += nb;
        items.push_back(it);
      }
    }
    for (int bl = 0; bl < nblk; ++bl) {
      RedBlock rb;
      std::memset(&rb, 0, sizeof rb);
      rb.orow = p.row0[t] + 16 * bl;
      rb.nv = std::min(16, T->N - 16 * bl);
      rb.k0 = (int)slot_idx.size();
      slot_idx.insert(slot_idx.end(), bslots[bl].begin(), bslots[bl].end());
      rb.k1 = (int)slot_idx.size();
      for (int q = 0; q < kRedInline && rb.k0 + q < rb.k1; ++q) rb.slot[q] = slot_idx[rb.k0 + q];
      rblocks.push_back(rb);
    }
  }

  // Hand the forward items out longest first (the persistent kernel takes
  // them in list order), so the last ones to finish are short.  Each item
  // keeps its partial slots, so the order does not change any result.
  {
    std::vector<double> cost(items.size());
    for (size_t k = 0; k < items.size(); ++k) {
      double c = 0;
      for (int sg = items[k].seg0; sg < items[k].seg1; ++sg) c += segs[sg].KE + 4.0;
      cost[k] = c * items[k].nblk;
    }
    std::vector<size_t> order(items.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    std::vector<FwdItem> sorted(items.size());
    for (size_t k = 0; k < order.size(); ++k) sorted[k] = items[order[k]];
    items.swap(sorted);
  }

  // ---- static work lists of the streaming hadronic forward: items go, in
  // the order above, to the least loaded of one workgroup per compute unit;
  // each workgroup walks its items' groups as one list of records.  Every
  // group must last kStreamW k-steps per wave, so that an LDS buffer is
  // released before the copy that reuses it is issued.
  int ncu = 0;
  FK_TRY_HIP(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  ncu = std::max(ncu, 1);
  std::vector<StreamSeg> srec;
  std::vector<int32_t> wgptr;
  p.grid_stream = 0;
  if (had && X >= kStreamWaves && !items.empty()) {
    int minT = 1 << 30;
    for (const auto &it : items)
      for (int sg = it.seg0; sg < it.seg1; ++sg) minT = std::min(minT, (segs[sg].KE + 3) / 4);
    if (minT * (X / kStreamWaves) >= kStreamW) {
      const int G = std::min<int>(ncu, (int)items.size());
      const int nal = (X + kStreamWaves - 1) / kStreamWaves;
      std::vector<std::vector<int>> lists(G);
      std::vector<std::pair<double, int>> heap;  // (load, workgroup), min-heap
      for (int g = 0; g < G; ++g) heap.push_back({0.0, g});
      auto cmp = [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
        return x.first != y.first ? x.first > y.first : x.second > y.second;
      };
      std::make_heap(heap.begin(), heap.end(), cmp);
      // cost in k-steps of the busiest wave: T per job, ceil(X/8) jobs per
      // record, about five k-steps per group change and eight per item for
      // the combine and write of its partial sums
      std::vector<double> icost(items.size()), load(G, 0.0);
      for (size_t k = 0; k < items.size(); ++k) {
        double cost = 8.0;
        for (int sg = items[k].seg0; sg < items[k].seg1; ++sg)
          cost += (double)((segs[sg].KE + 3) / 4) * nal + 5.0;
        icost[k] = cost;
        std::pop_heap(heap.begin(), heap.end(), cmp);
        lists[heap.back().second].push_back((int)k);
        heap.back().first += cost;
        load[heap.back().second] += cost;
        std::push_heap(heap.begin(), heap.end(), cmp);
      }
      rebalance(lists, load, icost);
      wgptr.push_back(0);
      for (int g = 0; g < G; ++g) {
        for (int k : lists[g]) {
          const FwdItem &it = items[k];
          const int nv0 = std::min(16, it.ndata - 16 * it.block0);
          const int nv1 = it.nblk > 1 ? std::min(16, it.ndata - 16 * (it.block0 + 1)) : 0;
          for (int sg = it.seg0; sg < it.seg1; ++sg) {
            const SegRef &sr = segs[sg];
            StreamSeg r;
            std::memset(&r, 0, sizeof r);
            r.a0 = sr.base + (size_t)it.block0 * X * 16 * sr.KE;
            r.a1 = nv1 ? r.a0 + (size_t)nv0 * sr.KE : nullptr;
            r.nv0 = nv0;
            r.nv1 = nv1;
            r.KE = sr.KE;
            r.T = (sr.KE + 3) / 4;
            r.flav = gd[sr.gdesc].a;
            r.last = sg == it.seg1 - 1;
            r.bop_off = gd[sr.gdesc].bop_off;
            r.slot = it.slot0;
            srec.push_back(r);
          }
        }
        wgptr.push_back((int32_t)srec.size());
      }
      // the plan keeps the stream kernel only if seven column tiles fit
      p.grid_stream = had_stream_lds_bytes(7, X, p.maxT_fwd) ? G : 0;
    }
  }

  // ---- streaming DIS forward: each table's blocks in ranges of about
  // 1/(8 ncu) of all blocks, one workgroup per range (several workgroups
  // share a compute unit: measured on a 2 GiB set, ranges of 1/(8 ncu) read
  // 5.9 TB/s, 1/(2 ncu) 5.1, 1/(32 ncu) 4.9)
  std::vector<DisGroupRef> dgroups;
  std::vector<DisStreamWG> dwgs;
  p.dis_chunk = 0;
  if (!had) {
    int ttot_max = 0;
    long total_blk = 0;
    for (auto *t : ts) total_blk += (t->N + 15) / 16;
    // at least kDisStreamMinBlk blocks per range: a workgroup stages the B
    // operands of all its table's groups before it streams, which a single
    // block does not amortise (measured on the DIS global workload, 400
    // blocks, R=100: 20.9 -> 16.4 us BF16 and 71 -> 43 us FP32 per step
    // with 4 instead of 1; 2 to 4 alike, 6 and 8 slower in FP32)
    const int target = (int)std::max<long>(
        kDisStreamMinBlk, std::min<long>(kDisStreamMaxBlk, (total_blk + 8 * ncu - 1) / (8 * ncu)));
    for (size_t t = 0; t < ts.size(); ++t) {
      const int g0 = (int)dgroups.size();
      int ttot = 0;
      for (int sg : segidx[t]) {
        DisGroupRef r;
        r.base = segs[sg].base;
        r.KE = segs[sg].KE;
        r.T = (segs[sg].KE + 3) / 4;
        r.bop_off = gd[segs[sg].gdesc].bop_off;
        dgroups.push_back(r);
        ttot += r.T;
      }
      ttot_max = std::max(ttot_max, ttot);
      const int nblk = (ts[t]->N + 15) / 16;
      const int nr = (nblk + target - 1) / target;
      for (int k = 0; k < nr; ++k) {
        DisStreamWG wgd;
        std::memset(&wgd, 0, sizeof wgd);
        wgd.g0 = g0;
        wgd.g1 = (int)dgroups.size();
        wgd.block0 = (int)((long)nblk * k / nr);
        wgd.nblk = (int)((long)nblk * (k + 1) / nr) - wgd.block0;
        wgd.ndata = ts[t]->N;
        wgd.orow0 = p.row0[t];
        wgd.ttot = ttot;
        if (wgd.nblk > 0) dwgs.push_back(wgd);
      }
    }
    p.dis_ttot_max = ttot_max;
    // one column width for every pass of the plan (see run_forward)
    for (int nt : {8, 7, 4})
      if (dis_stream_lds_bytes(nt, ttot_max)) {
        p.dis_chunk = 16 * nt;
        break;
      }
  }

  // ---- adjoint items and the CSR of partial rows per output row (a, x)
  std::vector<std::vector<int64_t>> rows_out((size_t)F * X);
  std::vector<HadAdjItem> hadj;
  std::vector<DisAdjItem> dadj;
  size_t apart_floats = 0;
  if (had) {
    double pairs = 0;
    for (auto *t : ts) pairs += (double)t->agroups.size() * ((t->N + 15) / 16);
    const int tb = std::max(1, (int)std::lround(pairs / 768.0));
    int slot = 0;
    for (size_t t = 0; t < ts.size(); ++t) {
      const Table *T = ts[t];
      const int nblk = (T->N + 15) / 16;
      for (size_t gi = 0; gi < T->agroups.size(); ++gi)
        for (int b0 = 0; b0 < nblk; b0 += tb) {
          HadAdjItem it;
          it.seg = asegidx[t][gi];
          it.block0 = b0;
          it.block1 = std::min(nblk, b0 + tb);
          it.ndata = T->N;
          it.wrow0 = p.row0[t];
          it.slot = slot;
          const int a = T->agroups[gi].a;
          for (int al = 0; al < X; ++al)
            rows_out[(size_t)a * X + al].push_back((int64_t)slot * X * kRpMax + (int64_t)al * kRpMax);
          ++slot;
          hadj.push_back(it);
        }
    }
    apart_floats = (size_t)slot * X * kRpMax;
  } else {
    int slot = 0;
    for (size_t t = 0; t < ts.size(); ++t) {
      const Table *T = ts[t];
      const int nrows = T->nact * X;
      const int ntile = (nrows + 15) / 16;
      for (size_t ch = 0; ch < T->tchunks.size(); ++ch) {
        const TChunk &tc = T->tchunks[ch];
        for (int q = 0; q < ntile; q += kWaves) {
          DisAdjItem it;
          it.base = (const uint4 *)((const char *)T->d_fkT + tc.base * 16);
          it.gdesc = chunkgd[t][ch];
          it.KE = tc.KE;
          it.nrows = nrows;
          it.tile0 = q;
          it.ntile = std::min(kWaves, ntile - q);
          it.slot0 = slot;
          for (int w = 0; w < it.ntile; ++w)
            for (int r = 0; r < 16; ++r) {
              const int lr = 16 * (q + w) + r;
              if (lr >= nrows) break;
              const int fl = T->active[lr / X], al = lr % X;
              rows_out[(size_t)fl * X + al].push_back((int64_t)(slot + w) * 16 * kRpMax +
                                                       (int64_t)r * kRpMax);
            }
          slot += it.ntile;
          dadj.push_back(it);
        }
      }
    }
    apart_floats = (size_t)slot * 16 * kRpMax;
  }
  std::vector<int32_t> row_ptr(1, 0);
  std::vector<int64_t> entries;
  for (auto &r : rows_out) {
    entries.insert(entries.end(), r.begin(), r.end());
    row_ptr.push_back((int32_t)entries.size());
  }

  // ---- streaming hadronic adjoint.  Items: one adjoint group of a table
  // over a run of kAdjPairsPerItem block pairs (a split that depends on the
  // table alone); records: one block pair of an item.  Each wave keeps the
  // gradient rows of its x indices in registers (at most 8 per wave, so
  // X <= 64), and every record must last kStreamW k-steps per wave.  The
  // weights gbar * s are staged per block pair (32 padded rows, zero past a
  // table's last datapoint), column by column.
  std::vector<StreamSeg> asrec;
  std::vector<int32_t> awgptr, wrow, row_ptr2(1, 0);
  std::vector<int64_t> entries2;
  size_t apart2_floats = 0;
  p.grid_astream = 0;
  if (had && X >= kStreamWaves && X <= 8 * kStreamWaves) {
    int minT = 1 << 30;
    for (auto *t : ts)
      for (auto &g : t->agroups) minT = std::min(minT, (g.KE + 3) / 4);
    if (minT < (1 << 30) && minT * (X / kStreamWaves) >= kStreamW &&
        had_stream_lds_bytes(7, X, p.maxT_adj, kStreamAdj)) {
      std::vector<int> pbase(ts.size());
      int nptot = 0;
      for (size_t t = 0; t < ts.size(); ++t) {
        pbase[t] = nptot;
        nptot += ((ts[t]->N + 15) / 16 + 1) / 2;
      }
      wrow.assign((size_t)nptot * 32, -1);
      for (size_t t = 0; t < ts.size(); ++t)
        for (int r = 0; r < ts[t]->N; ++r) wrow[(size_t)pbase[t] * 32 + r] = p.row0[t] + r;
      struct AItem {
        int t, gi, pair0, pair1, slot;
      };
      std::vector<AItem> aitems;
      std::vector<std::vector<int64_t>> rows2((size_t)F * X);
      int slot = 0;
      for (size_t t = 0; t < ts.size(); ++t) {
        const int npair = ((ts[t]->N + 15) / 16 + 1) / 2;
        for (size_t gi = 0; gi < ts[t]->agroups.size(); ++gi)
          for (int p0 = 0; p0 < npair; p0 += kAdjPairsPerItem) {
            aitems.push_back({(int)t, (int)gi, p0, std::min(npair, p0 + kAdjPairsPerItem), slot});
            const int a = ts[t]->agroups[gi].a;
            for (int al = 0; al < X; ++al)
              rows2[(size_t)a * X + al].push_back((int64_t)slot * X * kRpMax + (int64_t)al * kRpMax);
            ++slot;
          }
      }
      apart2_floats = (size_t)slot * X * kRpMax;
      for (auto &r : rows2) {
        entries2.insert(entries2.end(), r.begin(), r.end());
        row_ptr2.push_back((int32_t)entries2.size());
      }
      // cost in k-steps of the busiest wave, as for the forward lists
      const int nal = (X + kStreamWaves - 1) / kStreamWaves;
      std::vector<double> acost(aitems.size());
      for (size_t k = 0; k < aitems.size(); ++k) {
        const AItem &it = aitems[k];
        const SegRef &sr = segs[asegidx[it.t][it.gi]];
        acost[k] = 8.0 + (double)(it.pair1 - it.pair0) * ((double)((sr.KE + 3) / 4) * nal + 5.0);
      }
      const int G = std::min<int>(ncu, (int)aitems.size());
      const auto lists = partition_items(acost, G);
      awgptr.push_back(0);
      for (int g = 0; g < G; ++g) {
        for (int k : lists[g]) {
          const AItem &it = aitems[k];
          const Table *T = ts[it.t];
          const int nblk = (T->N + 15) / 16;
          const SegRef &sr = segs[asegidx[it.t][it.gi]];
          for (int pp = it.pair0; pp < it.pair1; ++pp) {
            const int bl0 = 2 * pp, bl1 = 2 * pp + 1;
            StreamSeg r;
            std::memset(&r, 0, sizeof r);
            r.nv0 = std::min(16, T->N - 16 * bl0);
            r.nv1 = bl1 < nblk ? std::min(16, T->N - 16 * bl1) : 0;
            r.a0 = sr.base + (size_t)bl0 * X * sr.KE * 16;
            r.a1 = r.nv1 ? sr.base + (size_t)bl1 * X * sr.KE * 16 : nullptr;
            r.KE = sr.KE;
            r.T = (sr.KE + 3) / 4;
            r.flav = pbase[it.t] + pp;
            r.last = pp == it.pair1 - 1;
            r.bop_off = gd[sr.gdesc].bop_off;
            r.slot = it.slot;
            asrec.push_back(r);
          }
        }
        awgptr.push_back((int32_t)asrec.size());
      }
      p.grid_astream = G;
    }
  }

  fk_status st;
  if ((st = upload(c, p, gd, &p.d_gd))) return st;
  if ((st = upload(c, p, rowtab, &p.d_rowtab))) return st;
  if ((st = upload(c, p, segs, &p.d_seg))) return st;
  if ((st = upload(c, p, items, &p.d_fitems))) return st;
  if ((st = upload(c, p, rblocks, &p.d_rblocks))) return st;
  if ((st = upload(c, p, slot_idx, &p.d_slot_idx))) return st;
  if ((st = upload(c, p, hadj, &p.d_hadj))) return st;
  if ((st = upload(c, p, dadj, &p.d_dadj))) return st;
  if ((st = upload(c, p, row_ptr, &p.d_arow_ptr))) return st;
  if ((st = upload(c, p, entries, &p.d_aentry))) return st;
  if ((st = upload(c, p, scale_all, &p.d_scale))) return st;
  if (p.grid_stream) {
    if ((st = upload(c, p, srec, &p.d_srec))) return st;
    if ((st = upload(c, p, wgptr, &p.d_wgptr))) return st;
  }
  if (p.grid_astream) {
    if ((st = upload(c, p, asrec, &p.d_asrec))) return st;
    if ((st = upload(c, p, awgptr, &p.d_awgptr))) return st;
    if ((st = upload(c, p, wrow, &p.d_wrow))) return st;
    if ((st = upload(c, p, row_ptr2, &p.d_arow_ptr2))) return st;
    if ((st = upload(c, p, entries2, &p.d_aentry2))) return st;
    p.nwpair = (int)(wrow.size() / 32);
  }
  if (p.dis_chunk) {
    if ((st = upload(c, p, dgroups, &p.d_dgroups))) return st;
    if ((st = upload(c, p, dwgs, &p.d_dwgs))) return st;
    p.n_dwgs = (int)dwgs.size();
  }
  p.nfitems = (int)items.size();
  p.nrblocks = (int)rblocks.size();
  p.nhadj = (int)hadj.size();
  p.ndadj = (int)dadj.size();
  void *d = nullptr;
  if ((st = dev_alloc(c, bop * 16, &d, &p.allocs))) return st;
  p.d_bop = (uint4 *)d;
  if ((st = dev_alloc(c, (size_t)nslots * 16 * kRpMax * 4, &d, &p.allocs))) return st;
  p.d_fpart = (float *)d;
  if ((st = dev_alloc(c, std::max(apart_floats, apart2_floats) * 4, &d, &p.allocs))) return st;
  p.d_apart = (float *)d;
  if (p.grid_astream) {
    if ((st = dev_alloc(c, (size_t)p.nwpair * kRpMax * kAdjWRow * 4, &d, &p.allocs))) return st;
    p.d_wstage = (float *)d;
  }
  if ((st = dev_alloc(c, kZeroPageBytes, &p.d_zero, &p.allocs))) return st;
  FK_TRY_HIP(c, hipMemset(p.d_zero, 0, kZeroPageBytes));
  if ((st = dev_alloc(c, 64, &d, &p.allocs))) return st;
  p.d_counter = (int *)d;
  FK_TRY_HIP(c, hipMemset(p.d_counter, 0, 64));
  if (p.grid_stream) {
    if ((st = dev_alloc(c, (size_t)F * X * kRpMax * 4, &d, &p.allocs))) return st;
    p.d_fstage = (float *)d;
  }
  p.grid_fwd = 2 * ncu;
  p.bop_units = bop;
  p.fpart_floats = (size_t)nslots * 16 * kRpMax;
  p.apart_floats = std::max(apart_floats, apart2_floats);
  p.bytes = 0;
  for (auto &a : p.allocs) p.bytes += a.second;
  return FK_OK;
}

hipEvent_t Timing::begin(hipStream_t s) {
  if (!on.load()) return nullptr;
  hipEvent_t a = nullptr;
  if (hipEventCreate(&a) != hipSuccess) return nullptr;
  (void)hipEventRecord(a, s);
  return a;
}

void Timing::end(int kind, hipEvent_t a, hipStream_t s) {
  if (!a) return;
  hipEvent_t b = nullptr;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return;
  }
  (void)hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(mu);
  pending.push_back({kind, a, b});
}

// Run ``launch`` bracketed by timing events of kind ``kind`` when enabled.
template <typename F>
static hipError_t timed(Timing *tm, int kind, hipStream_t s, F &&launch) {
  hipEvent_t a = tm ? tm->begin(s) : nullptr;
  hipError_t e = launch();
  if (tm) tm->end(kind, a, s);
  return e;
}

fk_status clone_forward_scratch(fk_ctx *c, const Plan &p, Plan &q,
                                std::vector<std::pair<void *, size_t>> *track) {
  q = p;
  q.allocs.clear();
  q.bytes = 0;
  q.d_apart = nullptr;
  q.d_wstage = nullptr;
  void *d = nullptr;
  fk_status st;
  if ((st = dev_alloc(c, std::max<size_t>(p.bop_units, 1) * 16, &d, track))) return st;
  q.d_bop = (uint4 *)d;
  if ((st = dev_alloc(c, std::max<size_t>(p.fpart_floats, 1) * 4, &d, track))) return st;
  q.d_fpart = (float *)d;
  if ((st = dev_alloc(c, 64, &d, track))) return st;
  q.d_counter = (int *)d;
  FK_TRY_HIP(c, hipMemset(q.d_counter, 0, 64));
  if (p.d_fstage) {
    if ((st = dev_alloc(c, (size_t)p.F * p.X * kRpMax * 4, &d, track))) return st;
    q.d_fstage = (float *)d;
  }
  return FK_OK;
}

hipError_t run_forward(const Plan &p, const float *pdf, int nrep, float *out, hipStream_t s,
                       Timing *tm, int kernels) {
  // FK_KERNELS_ITEM selects the persistent hadronic forward kernel (for
  // comparisons; the two kernels sum in different orders).  A plan that
  // uses the stream kernel uses it for every column pass, so that a
  // request's result does not depend on the replica count it is batched
  // with: passes are cut to 112 columns when 128 do not fit its LDS.
  const bool no_stream = kernels == FK_KERNELS_ITEM;
  const bool stream = p.kind == FK_HAD && p.grid_stream > 0 && !no_stream;
  const bool dstream = p.kind == FK_DIS && p.dis_chunk > 0 && !no_stream;
  const int chunk = dstream ? p.dis_chunk
                            : (stream && !had_stream_lds_bytes(8, p.X, p.maxT_fwd) ? 112 : kRpMax);
  for (int c0 = 0; c0 < nrep; c0 += chunk) {
    const int ncols = std::min(chunk, nrep - c0);
    ConvLaunch L{p.dtype, pick_nt(ncols), ncols, c0, nrep, s, p.d_zero};
    const int RP = 16 * L.nt;
    hipError_t e = timed(tm, FK_K_STAGE, s, [&] {
      return launch_stage_b(L, p.d_gd, p.d_rowtab, p.ngd_fwd, pdf, nullptr, p.d_scale, p.d_bop, p.d_counter,
                            stream ? p.d_fstage : nullptr, p.F, p.X);
    });
    if (e != hipSuccess) return e;
    if (dstream) {
      // the DIS stream kernel writes the output rows itself
      e = timed(tm, FK_K_DIS_STREAM, s, [&] {
        return launch_dis_stream(L, p.d_dwgs, p.n_dwgs, p.d_dgroups, p.d_bop, p.d_scale,
                                 p.dis_ttot_max, out);
      });
      if (e != hipSuccess) return e;
      continue;
    }
    if (stream)
      e = timed(tm, FK_K_HAD_STREAM, s, [&] {
        return launch_had_stream(L, p.d_srec, p.d_wgptr, p.grid_stream, p.d_bop, p.d_fstage, p.X,
                                 p.maxT_fwd, p.d_fpart);
      });
    else if (p.kind == FK_HAD)
      e = timed(tm, FK_K_HAD_FWD, s, [&] {
        return launch_had_fwd(L, p.d_fitems, p.nfitems, p.d_seg, p.d_gd, p.d_bop, pdf, p.X,
                              4 * p.maxT_fwd * RP, p.d_fpart, p.d_counter, p.grid_fwd);
      });
    else
      e = timed(tm, FK_K_DIS_FWD, s, [&] {
        return launch_dis_fwd(L, p.d_fitems, p.nfitems, p.d_seg, p.d_gd, p.d_bop,
                              4 * p.maxT_fwd * RP, p.d_fpart);
      });
    if (e != hipSuccess) return e;
    e = timed(tm, FK_K_FWD_REDUCE, s, [&] {
      return launch_fwd_reduce(L, p.d_rblocks, p.nrblocks, p.d_slot_idx, p.d_fpart, p.d_scale,
                               1.0f, out);
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_backward(const Plan &p, const float *pdf, const float *gout, int nrep, float *g,
                        int accumulate, hipStream_t s, Timing *tm, int kernels) {
  // The stream adjoint (when the plan has it) runs in passes of 112 columns
  // when 128 do not fit its LDS; FK_KERNELS_ITEM selects the per-item
  // kernel, as for the forward.
  const bool astream = p.kind == FK_HAD && p.grid_astream > 0 && kernels != FK_KERNELS_ITEM;
  const int chunk =
      astream && !had_stream_lds_bytes(8, p.X, p.maxT_adj, kStreamAdj) ? 112 : kRpMax;
  for (int c0 = 0; c0 < nrep; c0 += chunk) {
    const int ncols = std::min(chunk, nrep - c0);
    ConvLaunch L{p.dtype, pick_nt(ncols), ncols, c0, nrep, s, p.d_zero};
    const int RP = 16 * L.nt;
    hipError_t e;
    if (astream) {
      e = timed(tm, FK_K_STAGE, s, [&] {
        return launch_stage_b(L, p.d_gd + p.ngd_fwd, p.d_rowtab, p.ngd_adj, pdf, gout, p.d_scale,
                              p.d_bop, nullptr, nullptr, 0, 0, p.d_wrow, p.d_wstage, p.nwpair);
      });
      if (e != hipSuccess) return e;
      e = timed(tm, FK_K_HAD_ADJ_STREAM, s, [&] {
        return launch_had_stream(L, p.d_asrec, p.d_awgptr, p.grid_astream, p.d_bop, p.d_wstage,
                                 p.X, p.maxT_adj, p.d_apart, kStreamAdj);
      });
      if (e != hipSuccess) return e;
      e = timed(tm, FK_K_ADJ_REDUCE, s, [&] {
        return launch_adj_reduce(L, p.F * p.X, p.d_arow_ptr2, p.d_aentry2, p.d_apart, accumulate,
                                 g);
      });
      if (e != hipSuccess) return e;
      continue;
    }
    if (p.kind == FK_HAD) {
      e = timed(tm, FK_K_STAGE, s, [&] {
        return launch_stage_b(L, p.d_gd + p.ngd_fwd, p.d_rowtab, p.ngd_adj, pdf, nullptr, p.d_scale, p.d_bop,
                              nullptr);
      });
      if (e != hipSuccess) return e;
      e = timed(tm, FK_K_HAD_ADJ, s, [&] {
        return launch_had_adj(L, p.d_hadj, p.nhadj, p.d_seg, p.d_gd, p.d_bop, gout, p.d_scale,
                              p.X, 4 * p.maxT_adj * RP, p.d_apart);
      });
    } else {
      e = timed(tm, FK_K_STAGE, s, [&] {
        return launch_stage_b(L, p.d_gd + p.ngd_fwd, p.d_rowtab, p.ngd_adj, nullptr, gout, p.d_scale,
                              p.d_bop, nullptr);
      });
      if (e != hipSuccess) return e;
      e = timed(tm, FK_K_DIS_ADJ, s, [&] {
        return launch_dis_adj(L, p.d_dadj, p.ndadj, p.d_gd, p.d_bop, 4 * p.maxT_adj * RP,
                              p.d_apart);
      });
    }
    if (e != hipSuccess) return e;
    e = timed(tm, FK_K_ADJ_REDUCE, s, [&] {
      return launch_adj_reduce(L, p.F * p.X, p.d_arow_ptr, p.d_aentry, p.d_apart, accumulate, g);
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace fk

// ===========================================================================
// C entry points
// ===========================================================================
extern "C" {

fk_status fk_create(fk_ctx **out, int32_t device, uint64_t hbm_budget_bytes) {
  if (!out) return set_err(nullptr, FK_E_ARG, "fk_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0)
    return set_err(nullptr, FK_E_HIP, "fk_create: no HIP device (%s)", hipGetErrorString(e));
  if (device < 0 || device >= ndev)
    return set_err(nullptr, FK_E_ARG, "fk_create: device %d out of range [0,%d)", device, ndev);
  if ((e = hipSetDevice(device)) != hipSuccess)
    return set_err(nullptr, FK_E_HIP, "hipSetDevice: %s", hipGetErrorString(e));
  size_t fre = 0, tot = 0;
  if ((e = hipMemGetInfo(&fre, &tot)) != hipSuccess)
    return set_err(nullptr, FK_E_HIP, "hipMemGetInfo: %s", hipGetErrorString(e));
  // the device address of this GPU's static scratch (fk_conv_dis_static)
  if (device >= kMaxDevices || (e = static_scratch_resolve(device)) != hipSuccess)
    return set_err(nullptr, FK_E_HIP, "fk_create: static scratch of device %d: %s", device,
                   device >= kMaxDevices ? "device index too large" : hipGetErrorString(e));
  auto *c = new fk_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)fre);
  *out = c;
  return FK_OK;
}

fk_status fk_serve_stop(fk_ctx *ctx);

fk_status fk_destroy(fk_ctx *ctx) {
  if (!ctx) return FK_E_ARG;
  (void)hipSetDevice(ctx->device);
  fk_serve_stop(ctx);
  (void)hipDeviceSynchronize();
  for (auto &kv : ctx->plans) dev_free_all(ctx, kv.second->allocs);
  for (auto &kv : ctx->covs) dev_free_all(ctx, kv.second->allocs);
  for (auto &kv : ctx->mlps) dev_free_all(ctx, kv.second->allocs);
  for (auto &kv : ctx->tables) dev_free_all(ctx, kv.second->allocs);
  delete ctx;
  return FK_OK;
}

const char *fk_last_error(const fk_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

fk_status fk_memory(const fk_ctx *ctx, uint64_t *used_bytes, uint64_t *budget_bytes) {
  if (!ctx) return FK_E_ARG;
  if (used_bytes) *used_bytes = ctx->used.load();
  if (budget_bytes) *budget_bytes = ctx->budget;
  return FK_OK;
}

fk_status fk_set_option(fk_ctx *ctx, int32_t option, int64_t value) {
  if (!ctx) return FK_E_ARG;
  if (option == FK_OPT_KERNELS) {
    if (value != FK_KERNELS_STREAM && value != FK_KERNELS_ITEM)
      return set_err(ctx, FK_E_ARG, "fk_set_option: FK_OPT_KERNELS takes FK_KERNELS_STREAM or "
                     "FK_KERNELS_ITEM (got %lld)", (long long)value);
    ctx->kernels.store((int)value);
    return FK_OK;
  }
  return set_err(ctx, FK_E_ARG, "fk_set_option: unknown option %d", option);
}

fk_status fk_load_table(fk_ctx *ctx, int32_t kind, int32_t ndata, int32_t nflav, int32_t nx,
                        const double *xgrid, const uint8_t *mask, const double *fkv,
                        int32_t store_dtype, fk_table *out) {
  if (!ctx) return FK_E_ARG;
  Guard g(ctx);
  if (!out || !xgrid || !mask || !fkv)
    return set_err(ctx, FK_E_ARG, "fk_load_table: NULL pointer argument");
  *out = 0;
  if (kind != FK_DIS && kind != FK_HAD) return set_err(ctx, FK_E_ARG, "fk_load_table: bad kind %d", kind);
  if (store_dtype != FK_F32 && store_dtype != FK_BF16 && store_dtype != FK_FP8E4M3)
    return set_err(ctx, FK_E_ARG, "fk_load_table: bad store_dtype %d", store_dtype);
  if (ndata < 1 || nflav < 1 || nflav > 64 || nx < 2 || nx > kMaxNx)
    return set_err(ctx, FK_E_SHAPE, "fk_load_table: sizes out of range (ndata=%d nflav=%d nx=%d; "
                   "need ndata>=1, 1<=nflav<=64, 2<=nx<=%d)", ndata, nflav, nx, kMaxNx);
  for (int i = 0; i < nx; ++i)
    if (!(xgrid[i] > 0.0) || !std::isfinite(xgrid[i]) || (i && !(xgrid[i] > xgrid[i - 1])))
      return set_err(ctx, FK_E_GRID, "fk_load_table: x-grid must be positive and increasing");
  const int nm = kind == FK_DIS ? nflav : nflav * nflav;
  int nact = 0;
  for (int i = 0; i < nm; ++i) nact += mask[i] ? 1 : 0;
  if (nact == 0) return set_err(ctx, FK_E_SHAPE, "fk_load_table: mask has no active entry");
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  auto t = std::make_unique<Table>();
  t->kind = kind;
  t->N = ndata;
  t->F = nflav;
  t->X = nx;
  t->dtype = store_dtype;
  t->xgrid.assign(xgrid, xgrid + nx);
  PackedTable pt;
  try {
    if (kind == FK_DIS)
      pack_dis(fkv, mask, ndata, nflav, nx, store_dtype, pt);
    else
      pack_had(fkv, mask, ndata, nflav, nx, store_dtype, pt);
  } catch (const std::exception &ex) {
    return set_err(ctx, FK_E_HIP, "fk_load_table: packing failed: %s", ex.what());
  }
  std::vector<std::pair<void *, size_t>> track;
  fk_status st = dev_alloc(ctx, pt.fk.size(), &t->d_fk, &track);
  if (st) return st;
  t->fk_bytes = pt.fk.size();
  if (!pt.fkT.empty()) {
    if ((st = dev_alloc(ctx, pt.fkT.size(), &t->d_fkT, &track))) {
      dev_free_all(ctx, track);
      return st;
    }
    t->fkT_bytes = pt.fkT.size();
  }
  hipError_t e = hipMemcpy(t->d_fk, pt.fk.data(), pt.fk.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && t->d_fkT)
    e = hipMemcpy(t->d_fkT, pt.fkT.data(), pt.fkT.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dev_free_all(ctx, track);
    return set_err(ctx, FK_E_HIP, "fk_load_table: copy to device: %s", hipGetErrorString(e));
  }
  t->groups = std::move(pt.groups);
  t->agroups = std::move(pt.agroups);
  t->tchunks = std::move(pt.tchunks);
  t->active = std::move(pt.active);
  t->scale = std::move(pt.scale);
  t->nact = pt.nact;
  t->allocs = std::move(track);
  auto p = std::make_unique<Plan>();
  p->kind = kind;
  p->dtype = store_dtype;
  p->F = nflav;
  p->X = nx;
  p->tables = {0};
  std::vector<Table *> ts{t.get()};
  if ((st = build_plan(ctx, *p, ts))) {
    dev_free_all(ctx, p->allocs);
    dev_free_all(ctx, t->allocs);
    return st;
  }
  const int64_t id = ctx->next_id++;
  p->tables = {id};
  ctx->tables[id] = std::move(t);
  ctx->plans[id] = std::move(p);
  *out = id;
  return FK_OK;
}

fk_status fk_group_create(fk_ctx *ctx, int32_t ntables, const fk_table *tables, fk_table *out) {
  if (!ctx) return FK_E_ARG;
  Guard g(ctx);
  if (!out || !tables || ntables < 1) return set_err(ctx, FK_E_ARG, "fk_group_create: bad arguments");
  *out = 0;
  std::vector<Table *> ts;
  for (int i = 0; i < ntables; ++i) {
    Table *t = find_table(ctx, tables[i]);
    if (!t) return set_err(ctx, FK_E_HANDLE, "fk_group_create: table %lld is not loaded", (long long)tables[i]);
    ts.push_back(t);
  }
  for (auto *t : ts) {
    if (t->kind != ts[0]->kind || t->dtype != ts[0]->dtype || t->F != ts[0]->F || t->X != ts[0]->X)
      return set_err(ctx, FK_E_SHAPE, "fk_group_create: members differ in kind, dtype, nflav or nx");
    for (int k = 0; k < t->X; ++k)
      if (std::fabs(t->xgrid[k] - ts[0]->xgrid[k]) > 1e-12 * std::fabs(ts[0]->xgrid[k]))
        return set_err(ctx, FK_E_GRID, "fk_group_create: members use different x-grids");
  }
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  auto p = std::make_unique<Plan>();
  p->kind = ts[0]->kind;
  p->dtype = ts[0]->dtype;
  p->F = ts[0]->F;
  p->X = ts[0]->X;
  p->is_group = true;
  fk_status st = build_plan(ctx, *p, ts);
  if (st) {
    dev_free_all(ctx, p->allocs);
    return st;
  }
  p->tables.assign(tables, tables + ntables);
  for (auto *t : ts) t->group_refs++;
  const int64_t id = ctx->next_id++;
  ctx->plans[id] = std::move(p);
  *out = id;
  return FK_OK;
}

fk_status fk_unload_table(fk_ctx *ctx, fk_table table) {
  if (!ctx) return FK_E_ARG;
  Guard g(ctx);
  Plan *p = find_plan(ctx, table);
  if (!p) return set_err(ctx, FK_E_HANDLE, "fk_unload_table: unknown handle %lld", (long long)table);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (p->is_group) {
    for (auto h : p->tables)
      if (Table *t = find_table(ctx, h)) t->group_refs--;
    dev_free_all(ctx, p->allocs);
    ctx->plans.erase(table);
    return FK_OK;
  }
  Table *t = find_table(ctx, table);
  if (t && t->busy > 0)
    return set_err(ctx, FK_E_STATE, "fk_unload_table: table %lld has serving passes in flight",
                   (long long)table);
  if (t && t->group_refs > 0)
    return set_err(ctx, FK_E_STATE, "fk_unload_table: table %lld is used by %d group(s)",
                   (long long)table, t->group_refs);
  dev_free_all(ctx, p->allocs);
  ctx->plans.erase(table);
  if (t) {
    dev_free_all(ctx, t->allocs);
    ctx->tables.erase(table);
  }
  return FK_OK;
}

fk_status fk_table_probe(fk_ctx *ctx, fk_table table, const float *pdf, int32_t nrep, double tol,
                         double *err, void *stream) {
  if (!ctx) return FK_E_ARG;
  if (!pdf || !err || nrep < 1 || !(tol >= 0.0))
    return set_err(ctx, FK_E_ARG, "fk_table_probe: need pdf, err, nrep >= 1 and tol >= 0");
  *err = -1.0;
  Plan *p = nullptr, *pf = nullptr;
  Table *t = nullptr;
  {
    Guard g(ctx);
    t = find_table(ctx, table);
    if (!t) return set_err(ctx, FK_E_HANDLE, "fk_table_probe: %lld is not a loaded table", (long long)table);
    if (!t->fallback || !find_table(ctx, t->fallback))
      return set_err(ctx, FK_E_STATE, "fk_table_probe: table %lld has no FP32 fallback linked",
                     (long long)table);
    p = find_plan(ctx, table);
    pf = find_plan(ctx, t->fallback);
  }
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  const hipStream_t s = (hipStream_t)stream;
  const size_t ny = (size_t)t->N * nrep;
  std::vector<std::pair<void *, size_t>> tmp;
  void *d = nullptr;
  fk_status st = dev_alloc(ctx, ny * 2 * sizeof(float) + (size_t)nrep * 2 * sizeof(double), &d, &tmp);
  if (st) return st;
  float *y = (float *)d, *yf = y + ny;
  double *sums = (double *)(yf + ny);
  const int kern = ctx->kernels.load();
  hipError_t e = run_forward(*p, pdf, nrep, y, s, nullptr, kern);
  if (e == hipSuccess) e = run_forward(*pf, pdf, nrep, yf, s, nullptr, kern);
  if (e == hipSuccess) e = launch_col_err(y, yf, t->N, nrep, sums, s);
  std::vector<double> h((size_t)nrep * 2);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), sums, h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free_all(ctx, tmp);
  if (e != hipSuccess) return set_err(ctx, FK_E_HIP, "fk_table_probe: %s", hipGetErrorString(e));
  double worst = 0.0;
  for (int r = 0; r < nrep; ++r) {
    const double num = std::sqrt(h[2 * r]), den = std::sqrt(h[2 * r + 1]);
    // an all-zero reference column: any nonzero result is an infinite error
    const double v = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
    worst = std::max(worst, v);
  }
  {
    Guard g(ctx);
    if (Table *tt = find_table(ctx, table)) {
      tt->probe_err = worst;
      tt->route_fallback = worst > tol;
    }
  }
  *err = worst;
  return FK_OK;
}

fk_status fk_table_info(fk_ctx *ctx, fk_table table, int32_t *kind, int32_t *ndata, int32_t *nflav,
                        int32_t *nx, int32_t *store_dtype, uint64_t *device_bytes) {
  if (!ctx) return FK_E_ARG;
  Guard g(ctx);
  Plan *p = find_plan(ctx, table);
  if (!p) return set_err(ctx, FK_E_HANDLE, "fk_table_info: unknown handle %lld", (long long)table);
  if (kind) *kind = p->kind;
  if (ndata) *ndata = p->Ntot;
  if (nflav) *nflav = p->F;
  if (nx) *nx = p->X;
  if (store_dtype) *store_dtype = p->dtype;
  if (device_bytes) *device_bytes = p->bytes + (p->is_group ? 0 : p->table_bytes);
  return FK_OK;
}

static fk_status conv_common(fk_ctx *ctx, fk_table table, int kind, const double *pdf_xgrid,
                             const float *pdf, int32_t nrep, float *out, void *stream,
                             const char *name) {
  if (!ctx) return FK_E_ARG;
  Plan *p;
  {
    Guard g(ctx);
    p = find_plan(ctx, table);
    if (!p) return set_err(ctx, FK_E_HANDLE, "%s: unknown handle %lld", name, (long long)table);
    if (p->kind != kind)
      return set_err(ctx, FK_E_ARG, "%s: handle %lld holds %s tables", name, (long long)table,
                     p->kind == FK_DIS ? "DIS" : "hadronic");
    if (!pdf || !out) return set_err(ctx, FK_E_ARG, "%s: NULL pdf or out", name);
    if (nrep < 1) return set_err(ctx, FK_E_ARG, "%s: nrep must be >= 1 (got %d)", name, nrep);
    if (pdf_xgrid) {
      Table *t = find_table(ctx, p->tables[0]);
      for (int k = 0; t && k < p->X; ++k)
        if (!(std::fabs(pdf_xgrid[k] - t->xgrid[k]) <= 1e-12 * std::fabs(t->xgrid[k])))
          return set_err(ctx, FK_E_GRID, "%s: PDF x-grid differs from the table's at index %d", name, k);
    }
  }
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  hipError_t e = run_forward(*p, pdf, nrep, out, (hipStream_t)stream, &ctx->timing, ctx->kernels.load());
  if (e != hipSuccess) return set_err(ctx, FK_E_HIP, "%s: launch failed: %s", name, hipGetErrorString(e));
  return FK_OK;
}

fk_status fk_conv_dis(fk_ctx *ctx, fk_table table, const double *pdf_xgrid, const float *pdf,
                      int32_t nrep, float *out, void *stream) {
  return conv_common(ctx, table, FK_DIS, pdf_xgrid, pdf, nrep, out, stream, "fk_conv_dis");
}

fk_status fk_conv_had(fk_ctx *ctx, fk_table table, const double *pdf_xgrid, const float *pdf,
                      int32_t nrep, float *out, void *stream) {
  return conv_common(ctx, table, FK_HAD, pdf_xgrid, pdf, nrep, out, stream, "fk_conv_had");
}

fk_status fk_conv_dis_static(fk_ctx *ctx, fk_table table, const double *pdf_xgrid,
                             const float *pdf, int32_t nrep, float *out, void *stream) {
  if (!ctx) return FK_E_ARG;
  const Plan *p;
  {
    Guard g(ctx);
    p = find_plan(ctx, table);
    if (!p) return set_err(ctx, FK_E_HANDLE, "fk_conv_dis_static: unknown handle %lld", (long long)table);
    if (p->kind != FK_DIS)
      return set_err(ctx, FK_E_ARG, "fk_conv_dis_static: handle %lld holds hadronic tables", (long long)table);
    if (!pdf || !out) return set_err(ctx, FK_E_ARG, "fk_conv_dis_static: NULL pdf or out");
    if (nrep < 1) return set_err(ctx, FK_E_ARG, "fk_conv_dis_static: nrep must be >= 1 (got %d)", nrep);
    if (pdf_xgrid) {
      const Table *t = find_table(ctx, p->tables[0]);
      for (int k = 0; t && k < p->X; ++k)
        if (!(std::fabs(pdf_xgrid[k] - t->xgrid[k]) <= 1e-12 * std::fabs(t->xgrid[k])))
          return set_err(ctx, FK_E_GRID, "fk_conv_dis_static: PDF x-grid differs from the table's at index %d", k);
    }
    if (!p->dis_chunk)
      return set_err(ctx, FK_E_STATE, "fk_conv_dis_static: handle %lld does not use the streaming DIS "
                     "kernel (its B operand does not fit the kernel's LDS)", (long long)table);
    if (p->bop_units * 16 > kStaticScratchBytes)
      return set_err(ctx, FK_E_TOO_LARGE, "fk_conv_dis_static: the staged PDF operand needs %llu bytes, "
                     "the static scratch holds %llu", (unsigned long long)(p->bop_units * 16),
                     (unsigned long long)kStaticScratchBytes);
  }
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  uint4 *bop = (uint4 *)static_scratch(ctx->device);
  if (!bop) return set_err(ctx, FK_E_STATE, "fk_conv_dis_static: static scratch not resolved");
  const hipStream_t s = (hipStream_t)stream;
  // the DIS stream form of run_forward with the staged operand in the
  // static scratch: stage, then the stream kernel writes the outputs
  for (int c0 = 0; c0 < nrep; c0 += p->dis_chunk) {
    const int ncols = std::min(p->dis_chunk, nrep - c0);
    ConvLaunch L{p->dtype, pick_nt(ncols), ncols, c0, nrep, s, p->d_zero};
    hipError_t e = launch_stage_b(L, p->d_gd, p->d_rowtab, p->ngd_fwd, pdf, nullptr, p->d_scale, bop,
                                  nullptr);
    if (e == hipSuccess)
      e = launch_dis_stream(L, p->d_dwgs, p->n_dwgs, p->d_dgroups, bop, p->d_scale, p->dis_ttot_max, out);
    if (e != hipSuccess)
      return set_err(ctx, FK_E_HIP, "fk_conv_dis_static: launch failed: %s", hipGetErrorString(e));
  }
  return FK_OK;
}

fk_status fk_conv_backward(fk_ctx *ctx, fk_table table, const float *pdf, const float *grad_out,
                           int32_t nrep, float *grad_pdf, int32_t accumulate, void *stream) {
  if (!ctx) return FK_E_ARG;
  Plan *p;
  {
    Guard g(ctx);
    p = find_plan(ctx, table);
    if (!p) return set_err(ctx, FK_E_HANDLE, "fk_conv_backward: unknown handle %lld", (long long)table);
    if (!grad_out || !grad_pdf || (p->kind == FK_HAD && !pdf))
      return set_err(ctx, FK_E_ARG, "fk_conv_backward: NULL pointer argument");
    if (nrep < 1) return set_err(ctx, FK_E_ARG, "fk_conv_backward: nrep must be >= 1");
  }
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  hipError_t e = run_backward(*p, pdf, grad_out, nrep, grad_pdf, accumulate, (hipStream_t)stream,
                              &ctx->timing, ctx->kernels.load());
  if (e != hipSuccess)
    return set_err(ctx, FK_E_HIP, "fk_conv_backward: launch failed: %s", hipGetErrorString(e));
  return FK_OK;
}

// ---------------------------------------------------------------------------
// flattened form of Table 3
// ---------------------------------------------------------------------------
static int device_cus(fk_ctx *ctx) {
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || ncu < 1)
    ncu = 256;
  return ncu;
}

fk_status fk_luminosity(fk_ctx *ctx, int32_t nflav, int32_t nx, const uint8_t *mask,
                        const float *pdf, int32_t nrep, float *lum, void *stream) {
  if (!ctx) return FK_E_ARG;
  if (!mask || !pdf || !lum) return set_err(ctx, FK_E_ARG, "fk_luminosity: NULL pointer argument");
  if (nflav < 1 || nflav > 64 || nx < 1 || nrep < 1)
    return set_err(ctx, FK_E_SHAPE, "fk_luminosity: need 1 <= nflav <= 64, nx >= 1, nrep >= 1");
  FlatPairs pairs;
  pairs.n = 0;
  for (int a = 0; a < nflav; ++a)
    for (int b = 0; b < nflav; ++b)
      if (mask[a * nflav + b]) {
        if (pairs.n == kFlatMaxPairs)
          return set_err(ctx, FK_E_SHAPE, "fk_luminosity: more than %d active pairs", kFlatMaxPairs);
        pairs.ab[pairs.n++] = (int16_t)(a * 64 + b);
      }
  if (pairs.n == 0) return set_err(ctx, FK_E_SHAPE, "fk_luminosity: mask has no active pair");
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  const hipError_t e = launch_lumi(pairs, nx, nrep, pdf, lum, (hipStream_t)stream);
  if (e != hipSuccess) return set_err(ctx, FK_E_HIP, "fk_luminosity: launch failed: %s", hipGetErrorString(e));
  return FK_OK;
}

fk_status fk_flat_conv_workspace(fk_ctx *ctx, int64_t n, int64_t k, int64_t r, uint64_t *bytes) {
  if (!ctx) return FK_E_ARG;
  if (!bytes || n < 1 || k < 1 || r < 1)
    return set_err(ctx, FK_E_ARG, "fk_flat_conv_workspace: need bytes and n, k, r >= 1");
  *bytes = flat_plan(n, k, r, device_cus(ctx)).work_bytes;
  return FK_OK;
}

fk_status fk_flat_conv(fk_ctx *ctx, int64_t n, int64_t k, int64_t r, const float *fk, const float *lum,
                       float *out, void *work, uint64_t work_bytes, void *stream) {
  if (!ctx) return FK_E_ARG;
  if (!fk || !lum || !out || n < 1 || k < 1 || r < 1)
    return set_err(ctx, FK_E_ARG, "fk_flat_conv: need fk, lum, out and n, k, r >= 1");
  if (n > 65535LL * 16 || r > 65535LL * 64)
    return set_err(ctx, FK_E_SHAPE, "fk_flat_conv: need n <= %lld and r <= %lld", 65535LL * 16,
                   65535LL * 64);
  const FlatPlan p = flat_plan(n, k, r, device_cus(ctx));
  if (p.work_bytes > work_bytes || (p.work_bytes && !work))
    return set_err(ctx, FK_E_ARG, "fk_flat_conv: the workspace needs %llu bytes (got %llu)",
                   (unsigned long long)p.work_bytes, (unsigned long long)work_bytes);
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  const hipError_t e = launch_flat(p, n, k, r, fk, lum, out, (float *)work, (hipStream_t)stream);
  if (e != hipSuccess) return set_err(ctx, FK_E_HIP, "fk_flat_conv: launch failed: %s", hipGetErrorString(e));
  return FK_OK;
}

// ---------------------------------------------------------------------------
// network PDF and gradient descent (the steps either side of the convolution)
// ---------------------------------------------------------------------------
fk_status fk_mlp_create(fk_ctx *ctx, int32_t nflav, int32_t nx, const double *xgrid, int32_t h1,
                        int32_t h2, const double *pre_alpha, const double *pre_beta, fk_mlp *out,
                        int32_t *nparams) {
  if (!ctx) return FK_E_ARG;
  Guard g(ctx);
  if (!xgrid || !pre_alpha || !pre_beta || !out)
    return set_err(ctx, FK_E_ARG, "fk_mlp_create: NULL pointer argument");
  *out = 0;
  if (nflav < 1 || nflav > 64 || nx < 1 || nx > kMlpMaxNx || h1 < 1 || h1 > 64 || h2 < 1 || h2 > 64)
    return set_err(ctx, FK_E_SHAPE, "fk_mlp_create: need 1 <= nflav, h1, h2 <= 64 and 1 <= nx <= %d",
                   kMlpMaxNx);
  if (mlp_lds_bytes(nflav, nx, h1, h2, true) > kMlpMaxLds)
    return set_err(ctx, FK_E_SHAPE, "fk_mlp_create: a replica's parameters and activations need %zu "
                   "bytes of LDS (at most %zu)", mlp_lds_bytes(nflav, nx, h1, h2, true), kMlpMaxLds);
  for (int i = 0; i < nx; ++i)
    if (!(xgrid[i] > 0.0 && xgrid[i] <= 1.0))
      return set_err(ctx, FK_E_GRID, "fk_mlp_create: x-grid values must lie in (0, 1]");
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  std::vector<float> h((size_t)(2 + nflav) * nx);
  for (int i = 0; i < nx; ++i) {
    h[i] = (float)xgrid[i];
    h[nx + i] = (float)std::log(xgrid[i]);
  }
  for (int a = 0; a < nflav; ++a)
    for (int i = 0; i < nx; ++i)
      h[(size_t)(2 + a) * nx + i] =
          (float)(std::pow(xgrid[i], pre_alpha[a]) * std::pow(1.0 - xgrid[i], pre_beta[a]));
  auto m = std::make_unique<Mlp>();
  void *d = nullptr;
  fk_status st = dev_alloc(ctx, h.size() * sizeof(float), &d, &m->allocs);
  if (st) return st;
  hipError_t e = hipMemcpy(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dev_free_all(ctx, m->allocs);
    return set_err(ctx, FK_E_HIP, "fk_mlp_create: copy to device: %s", hipGetErrorString(e));
  }
  m->dev = MlpDev{nflav, nx, h1, h2, (const float *)d, (const float *)d + 2 * nx};
  const int64_t id = ctx->next_id++;
  ctx->mlps[id] = std::move(m);
  *out = id;
  if (nparams) *nparams = mlp_nparams(nflav, h1, h2);
  return FK_OK;
}

fk_status fk_mlp_destroy(fk_ctx *ctx, fk_mlp mlp) {
  if (!ctx) return FK_E_ARG;
  Guard g(ctx);
  auto it = ctx->mlps.find(mlp);
  if (it == ctx->mlps.end()) return set_err(ctx, FK_E_HANDLE, "fk_mlp_destroy: unknown handle %lld", (long long)mlp);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  dev_free_all(ctx, it->second->allocs);
  ctx->mlps.erase(it);
  return FK_OK;
}

static fk_status find_mlp(fk_ctx *ctx, fk_mlp mlp, MlpDev *out, const char *name) {
  Guard g(ctx);
  auto it = ctx->mlps.find(mlp);
  if (it == ctx->mlps.end()) return set_err(ctx, FK_E_HANDLE, "%s: unknown network handle %lld", name, (long long)mlp);
  *out = it->second->dev;
  return FK_OK;
}

fk_status fk_mlp_forward(fk_ctx *ctx, fk_mlp mlp, const float *params, int32_t nrep, float *pdf,
                         void *stream) {
  if (!ctx) return FK_E_ARG;
  if (!params || !pdf || nrep < 1) return set_err(ctx, FK_E_ARG, "fk_mlp_forward: need params, pdf, nrep >= 1");
  MlpDev m;
  fk_status st = find_mlp(ctx, mlp, &m, "fk_mlp_forward");
  if (st) return st;
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  const hipError_t e = launch_mlp_forward(m, params, nrep, pdf, (hipStream_t)stream);
  if (e != hipSuccess) return set_err(ctx, FK_E_HIP, "fk_mlp_forward: launch failed: %s", hipGetErrorString(e));
  return FK_OK;
}

fk_status fk_mlp_backward(fk_ctx *ctx, fk_mlp mlp, const float *params, const float *grad_pdf,
                          int32_t nrep, float *grad_params, void *stream) {
  if (!ctx) return FK_E_ARG;
  if (!params || !grad_pdf || !grad_params || nrep < 1)
    return set_err(ctx, FK_E_ARG, "fk_mlp_backward: need params, grad_pdf, grad_params, nrep >= 1");
  MlpDev m;
  fk_status st = find_mlp(ctx, mlp, &m, "fk_mlp_backward");
  if (st) return st;
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  const hipError_t e = launch_mlp_backward(m, params, grad_pdf, nrep, grad_params, (hipStream_t)stream);
  if (e != hipSuccess) return set_err(ctx, FK_E_HIP, "fk_mlp_backward: launch failed: %s", hipGetErrorString(e));
  return FK_OK;
}

fk_status fk_sgd_update(fk_ctx *ctx, float *params, const float *grad, int64_t n, float lr, void *stream) {
  if (!ctx) return FK_E_ARG;
  if (!params || !grad || n < 1) return set_err(ctx, FK_E_ARG, "fk_sgd_update: need params, grad, n >= 1");
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  const hipError_t e = launch_sgd(params, grad, n, lr, (hipStream_t)stream);
  if (e != hipSuccess) return set_err(ctx, FK_E_HIP, "fk_sgd_update: launch failed: %s", hipGetErrorString(e));
  return FK_OK;
}

// ---------------------------------------------------------------------------
// covariance and chi2
// ---------------------------------------------------------------------------
fk_status fk_load_covariance(fk_ctx *ctx, int32_t nblocks, const int32_t *block_n,
                             const double *cov, fk_cov *out) {
  if (!ctx) return FK_E_ARG;
  Guard g(ctx);
  if (!out || !block_n || !cov || nblocks < 1)
    return set_err(ctx, FK_E_ARG, "fk_load_covariance: bad arguments");
  *out = 0;
  auto cv = std::make_unique<Cov>();
  cv->nblocks = nblocks;
  std::vector<int64_t> off;
  std::vector<int32_t> roff, rtb, rtr;
  int64_t o = 0;
  int r = 0;
  for (int b = 0; b < nblocks; ++b) {
    const int n = block_n[b];
    if (n < 1 || n > 65536) return set_err(ctx, FK_E_SHAPE, "fk_load_covariance: block %d size %d", b, n);
    cv->n.push_back(n);
    off.push_back(o);
    roff.push_back(r);
    for (int r0 = 0; r0 < n; r0 += 32) {
      rtb.push_back(b);
      rtr.push_back(r0);
    }
    o += (int64_t)n * n;
    r += n;
    cv->maxn = std::max(cv->maxn, n);
  }
  cv->ntot = r;
  cv->nrt = (int)rtb.size();
  // split products: lower entries of row tile r cover k tiles [0, r], upper
  // entries the i tiles [r, nt); kChi2Split tiles per entry, more in large
  // blocks so that a row tile has at most eight entries (the partial
  // products then take at most 8 x 32 KiB per row tile)
  std::vector<int4> lw, uw;
  std::vector<int32_t> lptr(1, 0), uptr(1, 0);
  {
    int rt = 0;
    for (int b = 0; b < nblocks; ++b) {
      const int nt = (block_n[b] + 31) / 32;
      const int kc = std::max(kChi2Split, (nt + 7) / 8);
      for (int rr = 0; rr < nt; ++rr, ++rt) {
        for (int t0 = 0; t0 <= rr; t0 += kc)
          lw.push_back(make_int4(rt, t0, std::min(rr + 1, t0 + kc), (int)lw.size()));
        lptr.push_back((int32_t)lw.size());
        for (int t0 = rr; t0 < nt; t0 += kc)
          uw.push_back(make_int4(rt, t0, std::min(nt, t0 + kc), (int)uw.size()));
        uptr.push_back((int32_t)uw.size());
      }
    }
  }
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  std::vector<std::pair<void *, size_t>> tmp;
  void *d = nullptr;
  fk_status st;
  auto fail = [&](fk_status s) {
    dev_free_all(ctx, tmp);
    dev_free_all(ctx, cv->allocs);
    return s;
  };
  if ((st = dev_alloc(ctx, (size_t)o * 8, &d, &tmp))) return fail(st);
  double *d_a = (double *)d;
  if ((st = dev_alloc(ctx, (size_t)nblocks * 4, &d, &tmp))) return fail(st);
  int32_t *d_flag = (int32_t *)d;
  if ((st = dev_alloc(ctx, (size_t)o * 8, &d, &cv->allocs))) return fail(st);
  cv->d_linv = (double *)d;
  if ((st = dev_alloc(ctx, nblocks * 4, &d, &cv->allocs))) return fail(st);
  cv->d_n = (int32_t *)d;
  if ((st = dev_alloc(ctx, nblocks * 8, &d, &cv->allocs))) return fail(st);
  cv->d_off = (int64_t *)d;
  if ((st = dev_alloc(ctx, nblocks * 4, &d, &cv->allocs))) return fail(st);
  cv->d_roff = (int32_t *)d;
  if ((st = dev_alloc(ctx, rtb.size() * 4, &d, &cv->allocs))) return fail(st);
  cv->d_rt_block = (int32_t *)d;
  if ((st = dev_alloc(ctx, rtr.size() * 4, &d, &cv->allocs))) return fail(st);
  cv->d_rt_row = (int32_t *)d;
  if ((st = dev_alloc(ctx, (size_t)cv->ntot * kRpMax * 8, &d, &cv->allocs))) return fail(st);
  cv->d_y = (double *)d;
  if ((st = dev_alloc(ctx, (size_t)cv->nrt * kRpMax * 8, &d, &cv->allocs))) return fail(st);
  cv->d_part = (double *)d;
  Chi2Plan &P = cv->plan;
  P.nrt = cv->nrt;
  P.nlw = (int)lw.size();
  P.nuw = (int)uw.size();
  if ((st = dev_alloc(ctx, (size_t)std::max(P.nlw, P.nuw) * 32 * kRpMax * 8, &d, &cv->allocs)))
    return fail(st);
  P.d_spart = (double *)d;
  int4 *d_lw = nullptr, *d_uw = nullptr;
  int32_t *d_lptr = nullptr, *d_uptr = nullptr;
  if ((st = dev_alloc(ctx, lw.size() * sizeof(int4), &d, &cv->allocs))) return fail(st);
  d_lw = (int4 *)d;
  if ((st = dev_alloc(ctx, uw.size() * sizeof(int4), &d, &cv->allocs))) return fail(st);
  d_uw = (int4 *)d;
  if ((st = dev_alloc(ctx, lptr.size() * 4, &d, &cv->allocs))) return fail(st);
  d_lptr = (int32_t *)d;
  if ((st = dev_alloc(ctx, uptr.size() * 4, &d, &cv->allocs))) return fail(st);
  d_uptr = (int32_t *)d;
  P.d_lw = d_lw;
  P.d_uw = d_uw;
  P.d_lptr = d_lptr;
  P.d_uptr = d_uptr;
  P.d_y = cv->d_y;
  P.d_part = cv->d_part;
  P.d_rt_block = cv->d_rt_block;
  P.d_rt_row = cv->d_rt_row;
  P.d_n = cv->d_n;
  P.d_roff = cv->d_roff;
  P.d_off = cv->d_off;
  hipError_t e = hipMemcpy(d_a, cov, (size_t)o * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(cv->d_n, cv->n.data(), nblocks * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(cv->d_off, off.data(), nblocks * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(cv->d_roff, roff.data(), nblocks * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(cv->d_rt_block, rtb.data(), rtb.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(cv->d_rt_row, rtr.data(), rtr.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_lw, lw.data(), lw.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_uw, uw.data(), uw.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_lptr, lptr.data(), lptr.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_uptr, uptr.data(), uptr.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(cv->d_linv, 0, (size_t)o * 8);
  if (e == hipSuccess) e = hipMemset(d_flag, 0, nblocks * 4);
  if (e == hipSuccess)
    e = launch_cholesky(nblocks, cv->d_n, cv->d_off, d_a, cv->d_linv, d_flag, cv->maxn, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  std::vector<int32_t> flags(nblocks, 0);
  if (e == hipSuccess) e = hipMemcpy(flags.data(), d_flag, nblocks * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    set_err(ctx, FK_E_HIP, "fk_load_covariance: %s", hipGetErrorString(e));
    return fail(FK_E_HIP);
  }
  for (int b = 0; b < nblocks; ++b)
    if (flags[b]) {
      set_err(ctx, FK_E_NOTPD, "fk_load_covariance: block %d is not positive definite (pivot %d)",
              b, flags[b] - 1);
      return fail(FK_E_NOTPD);
    }
  dev_free_all(ctx, tmp);
  cv->bytes = 0;
  for (auto &a : cv->allocs) cv->bytes += a.second;
  const int64_t id = ctx->next_id++;
  ctx->covs[id] = std::move(cv);
  *out = id;
  return FK_OK;
}

fk_status fk_unload_covariance(fk_ctx *ctx, fk_cov cov) {
  if (!ctx) return FK_E_ARG;
  Guard g(ctx);
  auto it = ctx->covs.find(cov);
  if (it == ctx->covs.end()) return set_err(ctx, FK_E_HANDLE, "fk_unload_covariance: unknown handle");
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  dev_free_all(ctx, it->second->allocs);
  ctx->covs.erase(it);
  return FK_OK;
}

fk_status fk_chi2(fk_ctx *ctx, fk_cov cov, const float *sigma, const double *data, int32_t nrep,
                  double *chi2, float *dchi2_dsigma, void *stream) {
  if (!ctx) return FK_E_ARG;
  Cov *cv;
  {
    Guard g(ctx);
    auto it = ctx->covs.find(cov);
    if (it == ctx->covs.end()) return set_err(ctx, FK_E_HANDLE, "fk_chi2: unknown covariance handle");
    cv = it->second.get();
    if (!sigma || !data || !chi2) return set_err(ctx, FK_E_ARG, "fk_chi2: NULL pointer argument");
    if (nrep < 1) return set_err(ctx, FK_E_ARG, "fk_chi2: nrep must be >= 1");
  }
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  for (int c0 = 0; c0 < nrep; c0 += kRpMax) {
    const int ncols = std::min(kRpMax, nrep - c0);
    hipEvent_t ta = ctx->timing.begin((hipStream_t)stream);
    hipError_t e = launch_chi2(cv->plan, cv->d_linv, sigma, data, nrep, c0, ncols, chi2,
                               dchi2_dsigma, (hipStream_t)stream);
    ctx->timing.end(FK_K_CHI2, ta, (hipStream_t)stream);
    if (e != hipSuccess) return set_err(ctx, FK_E_HIP, "fk_chi2: launch failed: %s", hipGetErrorString(e));
  }
  return FK_OK;
}

fk_status fk_timing_enable(fk_ctx *ctx, int32_t enable) {
  if (!ctx) return FK_E_ARG;
  ctx->timing.on = enable != 0;
  return FK_OK;
}

fk_status fk_timing_read(fk_ctx *ctx, double *total_ms, int64_t *launches) {
  if (!ctx) return FK_E_ARG;
  FK_TRY_HIP(ctx, hipSetDevice(ctx->device));
  Timing &T = ctx->timing;
  std::lock_guard<std::mutex> lk(T.mu);
  hipError_t err = hipSuccess;
  for (auto &r : T.pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e == hipSuccess) {
      T.total[r.kind] += ms;
      T.count[r.kind] += 1;
    } else if (err == hipSuccess) {
      err = e;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  T.pending.clear();
  for (int k = 0; k < FK_K_COUNT; ++k) {
    if (total_ms) total_ms[k] = T.total[k];
    if (launches) launches[k] = T.count[k];
    T.total[k] = 0.0;
    T.count[k] = 0;
  }
  if (err != hipSuccess) return set_err(ctx, FK_E_HIP, "fk_timing_read: %s", hipGetErrorString(err));
  return FK_OK;
}

}  // extern "C"
