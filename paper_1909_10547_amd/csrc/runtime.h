// Host runtime of the fkconv library: context, device-memory budget, table
// registry and launch plans.
#pragma once

#include <atomic>
#include <cstdarg>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fk_internal.h"
#include "pack.h"

struct fk_serve;  // serving loop (serve.cpp)

namespace fk {

// A loaded dataset.
struct Table {
  int kind = 0, N = 0, F = 0, X = 0, dtype = 0;
  std::vector<double> xgrid;
  std::vector<GroupPlan> groups;   // forward row groups (into d_fk)
  std::vector<GroupPlan> agroups;  // hadronic adjoint row groups (into d_fkT)
  std::vector<TChunk> tchunks;     // DIS adjoint chunks (into d_fkT)
  std::vector<int> active;
  std::vector<float> scale;
  int nact = 0;
  void *d_fk = nullptr, *d_fkT = nullptr;
  size_t fk_bytes = 0, fkT_bytes = 0;
  int64_t fallback = 0;
  int group_refs = 0;
  int busy = 0;  // serving passes in flight on this table
  // BF16/FP8 probe against the FP32 fallback (fk_table_probe): the measured
  // error, and whether requests for the table's own format go to the fallback
  double probe_err = -1.0;
  bool route_fallback = false;
  std::vector<std::pair<void *, size_t>> allocs;
};

// Everything one conv/backward call on a table or a group needs.
struct Plan {
  int kind = 0, dtype = 0, F = 0, X = 0, Ntot = 0;
  bool is_group = false;
  std::vector<int64_t> tables;
  std::vector<int> row0;
  // device descriptors
  GroupDesc *d_gd = nullptr;
  int32_t *d_rowtab = nullptr;  // gather rows of the descriptors (GroupDesc::row_off)
  int ngd_fwd = 0, ngd_adj = 0;  // forward descriptors, then adjoint-only ones
  SegRef *d_seg = nullptr;
  FwdItem *d_fitems = nullptr;
  int nfitems = 0;
  RedBlock *d_rblocks = nullptr;
  int nrblocks = 0;
  int32_t *d_slot_idx = nullptr;
  HadAdjItem *d_hadj = nullptr;
  int nhadj = 0;
  DisAdjItem *d_dadj = nullptr;
  int ndadj = 0;
  int32_t *d_arow_ptr = nullptr;
  int64_t *d_aentry = nullptr;
  float *d_scale = nullptr;
  // scratch
  uint4 *d_bop = nullptr;
  float *d_fpart = nullptr, *d_apart = nullptr;
  void *d_zero = nullptr;  // kZeroPageBytes of zeros read by lanes outside a tile
  int *d_counter = nullptr;  // work counter of the persistent forward kernel
  int grid_fwd = 512;        // persistent workgroups (2 per compute unit)
  // streaming hadronic forward: per-workgroup segment records
  StreamSeg *d_srec = nullptr;
  int32_t *d_wgptr = nullptr;
  int grid_stream = 0;        // 0: the plan does not use the stream kernel
  float *d_fstage = nullptr;  // [F][X][RP] FP32 PDF rows of the epilogue
  // streaming hadronic adjoint: its own records, items and CSR of slots
  StreamSeg *d_asrec = nullptr;
  int32_t *d_awgptr = nullptr;
  int grid_astream = 0;       // 0: the plan uses the per-item adjoint kernel
  int32_t *d_wrow = nullptr;  // [pair][32] padded weight row -> output row (-1: padding)
  int nwpair = 0;
  float *d_wstage = nullptr;  // [pair][RP][kAdjWRow] weights gbar * s
  int32_t *d_arow_ptr2 = nullptr;
  int64_t *d_aentry2 = nullptr;
  // streaming DIS forward
  DisGroupRef *d_dgroups = nullptr;
  DisStreamWG *d_dwgs = nullptr;
  int n_dwgs = 0;
  int dis_ttot_max = 0;
  int dis_chunk = 0;  // columns per pass of the DIS stream kernel; 0: not used
  int maxT_fwd = 1, maxT_adj = 1;
  // scratch sizes (for copies of the plan with private scratch)
  size_t bop_units = 0, fpart_floats = 0, apart_floats = 0;
  // bookkeeping
  std::vector<std::pair<void *, size_t>> allocs;
  uint64_t bytes = 0;
  uint64_t table_bytes = 0;  // device bytes of the member tables
};

// Optional per-kernel timing with event pairs on the launch stream.
struct Timing {
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::mutex mu;
  std::atomic<bool> on{false};
  std::vector<Rec> pending;
  double total[FK_K_COUNT] = {};
  int64_t count[FK_K_COUNT] = {};
  // bracket one launch: begin() before, end() after
  hipEvent_t begin(hipStream_t s);
  void end(int kind, hipEvent_t a, hipStream_t s);
};

struct Cov {
  int nblocks = 0, ntot = 0, maxn = 0, nrt = 0;
  std::vector<int> n;
  double *d_linv = nullptr;
  int32_t *d_n = nullptr, *d_roff = nullptr, *d_rt_block = nullptr, *d_rt_row = nullptr;
  int64_t *d_off = nullptr;
  double *d_y = nullptr, *d_part = nullptr;
  Chi2Plan plan;  // device pointers of the per-call work
  std::vector<std::pair<void *, size_t>> allocs;
  uint64_t bytes = 0;
};

struct Mlp {
  MlpDev dev;
  std::vector<std::pair<void *, size_t>> allocs;
};

}  // namespace fk

struct fk_ctx {
  int device = 0;
  uint64_t budget = 0;
  std::atomic<uint64_t> used{0};
  std::mutex mu;           // registry and error string
  std::string err;
  int64_t next_id = 1;
  std::map<int64_t, std::unique_ptr<fk::Table>> tables;
  std::map<int64_t, std::unique_ptr<fk::Plan>> plans;  // table handles and group handles
  std::map<int64_t, std::unique_ptr<fk::Cov>> covs;
  std::map<int64_t, std::unique_ptr<fk::Mlp>> mlps;
  fk_serve *serve = nullptr;
  fk::Timing timing;
  std::atomic<int> kernels{FK_KERNELS_STREAM};  // fk_set_option(FK_OPT_KERNELS)
};

namespace fk {

fk_status set_err(fk_ctx *c, fk_status code, const char *fmt, ...);
fk_status dev_alloc(fk_ctx *c, size_t bytes, void **p, std::vector<std::pair<void *, size_t>> *track);
void dev_free_all(fk_ctx *c, std::vector<std::pair<void *, size_t>> &track);
Plan *find_plan(fk_ctx *c, int64_t h);
Table *find_table(fk_ctx *c, int64_t h);

// Launch the forward or the adjoint of ``plan`` (no validation, no locking).
// ``kernels`` is FK_KERNELS_STREAM or FK_KERNELS_ITEM (fk_set_option).
hipError_t run_forward(const Plan &p, const float *pdf, int nrep, float *out, hipStream_t s,
                       Timing *tm = nullptr, int kernels = FK_KERNELS_STREAM);
hipError_t run_backward(const Plan &p, const float *pdf, const float *gout, int nrep, float *g,
                        int accumulate, hipStream_t s, Timing *tm = nullptr,
                        int kernels = FK_KERNELS_STREAM);
// A copy of ``p`` that shares its descriptors and table data but owns new
// forward scratch (tracked in ``track``), so that its forward passes can run
// concurrently with those of ``p``.  The copy has no adjoint scratch.
fk_status clone_forward_scratch(fk_ctx *c, const Plan &p, Plan &q,
                                std::vector<std::pair<void *, size_t>> *track);
int pick_nt(int ncols);

}  // namespace fk
