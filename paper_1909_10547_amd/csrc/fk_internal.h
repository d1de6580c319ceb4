// Internal declarations of the fkconv library: device descriptors shared by
// the host runtime and the kernels, and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fkconv.h"

namespace fk {

// ---------------------------------------------------------------------------
// Tiling constants
//
// Every kernel is a 16-row x (16*NT)-column MFMA tile computed by one wave64.
// The FK operand is stored in 16-byte "units"; one unit holds E consecutive
// contraction elements of one row (E = 4 float, 8 bfloat16, 16 e4m3).  A
// k-step is 4 units per row: lane (g = lane/16, row = lane%16) supplies unit
// 4t+g of row ``row``; the B operand (PDF, or the adjoint weights) lives in
// LDS in the same unit layout [unit][column].
// ---------------------------------------------------------------------------
constexpr int kWaves = 4;                  // waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kRpMax = 128;                // replica columns per pass
constexpr int kUnitsMax = 32;              // units per row and group (LDS B <= 64 KiB)
constexpr int kTMax = kUnitsMax / 4;       // k-steps per tile
constexpr int kMaxSeg = 40;                // segments per group descriptor
constexpr int kMaxNx = 128;                // grid points supported
constexpr int kDisChunkUnits = kUnitsMax;  // datapoint units per DIS adjoint chunk
constexpr int kItemUnits = 48;             // forward work per item (units per row)

inline int elems_per_unit(int dtype) {
  return dtype == FK_F32 ? 4 : (dtype == FK_BF16 ? 8 : 16);
}
inline int elem_bytes(int dtype) { return dtype == FK_F32 ? 4 : (dtype == FK_BF16 ? 2 : 1); }

// B-operand descriptor: the contraction index k of a group is the
// concatenation of ``nseg`` segments; segment s covers source rows
// seg_row[s] .. seg_row[s]+seg_len[s]-1.  Source 0 is the PDF (row =
// flavour*nx + x index), source 1 the adjoint weights gbar[i]*s_i (row =
// datapoint index in the concatenated output).
struct GroupDesc {
  int32_t a;        // row flavour of a hadronic group, -1 otherwise
  int32_t src;      // 0: PDF, 1: adjoint weights
  int32_t nseg;
  int32_t K;        // contraction length (sum of seg_len)
  int32_t KE;       // units per row = ceil(K / E)
  int32_t pad;
  int64_t bop_off;  // offset of the staged B operand, in 16-byte units
  int64_t row_off;  // offset of its gather rows: KEpad*E source rows, -1 past K
  int32_t seg_row[kMaxSeg];
  int32_t seg_len[kMaxSeg];
};

// One (table, group) of a plan: where the group's packed FK starts.
struct SegRef {
  const uint4 *base;
  int32_t gdesc;
  int32_t KE;
};

// Forward work item.  Hadronic: up to two 16-datapoint blocks, groups
// [seg0, seg1) of one table, waves split the x index alpha.  DIS: up to
// kWaves consecutive blocks (one per wave), groups [seg0, seg1).
struct FwdItem {
  int32_t seg0, seg1;
  int32_t block0;   // first block of the item within the table
  int32_t nblk;     // blocks in the item (DIS <= kWaves, hadronic <= 2)
  int32_t ndata;    // datapoints of the table
  int32_t slot0;    // first partial slot (16 x RP floats each)
};

// Segment record of the streaming hadronic forward: one group of one item
// in a workgroup's static work list (items in list order, groups in order).
struct StreamSeg {
  const uint4 *a0;    // block 0 of the item: packed group tile at alpha = 0
  const uint4 *a1;    // block 1, nullptr when the item has one block
  int32_t nv0, nv1;   // rows of the two blocks (nv1 = 0: absent)
  int32_t KE, T;      // units per row, k-steps (ceil(KE / 4))
  int32_t flav;       // forward: row flavour a, the PDF row of the epilogue;
                      // adjoint: first row of the pair in the padded weights
  int32_t last;       // 1 on the item's last group: write its partial sums
  int64_t bop_off;    // staged B operand of the group, in 16-byte units
  int32_t slot;       // first partial slot of the item
  int32_t pad;
};
constexpr int kAdjWaves = 8;      // waves per workgroup of the hadronic adjoint (x split 8 ways)
constexpr int kStreamW = 8;       // k-steps in flight per wave in the stream kernel
constexpr int kStreamWaves = 8;   // waves per workgroup of the stream kernel (2 per SIMD)
constexpr int kStreamFwd = 0;     // stream kernel modes: forward (PDF-row epilogue) ...
constexpr int kStreamAdj = 1;     // ... and adjoint (weighted row sums, gradient rows)
constexpr int kAdjPairsPerItem = 4;  // block pairs per item of the stream adjoint
constexpr int kAdjWRow = 36;  // floats per column of a pair's staged weights (32 rows + pad)

// DIS stream kernel: one group of a table (forward groups in k order).
struct DisGroupRef {
  const uint4 *base;  // packed group, block 0
  int32_t KE, T;      // units per row, k-steps
  int64_t bop_off;    // staged B operand (16-byte units)
};

// DIS stream kernel: one workgroup's range of 16-datapoint blocks of one
// table; the table's groups are [g0, g1) of the plan's DisGroupRef list.
struct DisStreamWG {
  int32_t g0, g1;
  int32_t block0, nblk;  // blocks of the table
  int32_t ndata;         // datapoints of the table
  int32_t orow0;         // output row of the table's datapoint 0
  int32_t ttot;          // k-steps per block over all groups
  int32_t pad;
};
constexpr int kDisStreamW = 16;      // k-steps in flight per wave
constexpr int kDisStreamWaves = 8;   // waves per workgroup
constexpr int kDisStreamMaxBlk = 512;  // blocks per workgroup (scales kept in LDS)
constexpr int kDisStreamMinBlk = 4;    // blocks per workgroup at least (amortise the B staging)

// Hadronic adjoint item: one group, blocks [block0, block1) of its table.
struct HadAdjItem {
  int32_t seg;
  int32_t block0, block1;
  int32_t ndata;
  int32_t wrow0;    // row of the table's datapoint 0 in the concatenated output
  int32_t slot;     // partial slot (nx x RP floats)
};

// DIS adjoint item on the transposed table: rows (flavour, x) in 16-row
// tiles, contraction over one chunk of datapoints.
struct DisAdjItem {
  const uint4 *base;  // packed transposed FK of the chunk, tile 0
  int32_t gdesc;      // B operand (weights of the chunk's datapoints)
  int32_t KE;
  int32_t nrows;      // nact * nx
  int32_t tile0;      // first 16-row tile of the item
  int32_t ntile;      // tiles in the item (<= kWaves)
  int32_t slot0;      // first partial slot (16 x RP floats each)
};

// Forward reduction of one output block of 16 datapoints.
constexpr int kRedInline = 8;  // slots of an output block held in its record
struct RedBlock {
  int32_t orow;     // first output row
  int32_t nv;       // rows in the block
  int32_t k0, k1;   // range in the slot index list
  int32_t slot[kRedInline];  // slot_idx[k0 .. k0 + kRedInline), where present
};

// ---------------------------------------------------------------------------
// Kernel launchers (conv_kernels.hip)
// ---------------------------------------------------------------------------
struct ConvLaunch {
  int dtype;
  int nt;           // column tiles of 16 (RP = 16*nt)
  int ncols, c0, R; // columns of this pass, their offset, caller's row stride
  hipStream_t stream;
  const void *zero_page;  // kZeroPageBytes of zeros in device memory
};
constexpr int kZeroPageBytes = 4096;

// Stages the B operands of ``ngd`` descriptors; with ``fstage`` also the
// FP32 PDF rows [nflav][nx][RP]; with ``wstage`` also the adjoint weights
// of ``nwpair`` block pairs, [pair][RP][kAdjWRow]: element (P, n, q) =
// gout[wrow[32 P + q]][c0 + n] * s, zero where wrow < 0, q >= 32 or n >= ncols.
hipError_t launch_stage_b(const ConvLaunch &L, const GroupDesc *d_gd, const int32_t *rowtab,
                          int ngd, const float *pdf,
                          const float *gout, const float *scale_all, uint4 *bop, int *counter,
                          float *fstage = nullptr, int nflav = 0, int nx = 0,
                          const int32_t *wrow = nullptr, float *wstage = nullptr, int nwpair = 0);
// LDS of the stream kernel for (nt, nx, maxT); 0 when it does not fit.
size_t had_stream_lds_bytes(int nt, int nx, int maxT, int mode = kStreamFwd);
// Stream kernel.  Forward: fstage = FP32 PDF rows [F][nx][RP], part =
// partial slots [slot][16][kRpMax].  Adjoint: fstage = the staged weights
// [pair][RP][kAdjWRow], part = gradient slots [slot][nx][kRpMax]; nx <= 64.
hipError_t launch_had_stream(const ConvLaunch &L, const StreamSeg *recs, const int32_t *wg_ptr,
                             int grid, const uint4 *bop, const float *fstage, int nx, int maxT,
                             float *part, int mode = kStreamFwd);
hipError_t launch_had_fwd(const ConvLaunch &L, const FwdItem *items, int nitems, const SegRef *segs,
                          const GroupDesc *gd, const uint4 *bop, const float *pdf, int nx,
                          int lds_units, float *part, int *counter, int grid);
// LDS of the DIS stream kernel for (nt, max k-steps per block); 0 when it
// does not fit.
size_t dis_stream_lds_bytes(int nt, int ttot_max);
hipError_t launch_dis_stream(const ConvLaunch &L, const DisStreamWG *wgs, int nwg,
                             const DisGroupRef *groups, const uint4 *bop, const float *scale_all,
                             int ttot_max, float *out);
hipError_t launch_dis_fwd(const ConvLaunch &L, const FwdItem *items, int nitems, const SegRef *segs,
                          const GroupDesc *gd, const uint4 *bop, int lds_units, float *part);
hipError_t launch_fwd_reduce(const ConvLaunch &L, const RedBlock *blocks, int nblocks,
                             const int32_t *slot_idx, const float *part, const float *scale_all,
                             float factor, float *out);
hipError_t launch_had_adj(const ConvLaunch &L, const HadAdjItem *items, int nitems,
                          const SegRef *segs, const GroupDesc *gd, const uint4 *bop,
                          const float *gout, const float *scale_all, int nx, int lds_units,
                          float *apart);
hipError_t launch_dis_adj(const ConvLaunch &L, const DisAdjItem *items, int nitems,
                          const GroupDesc *gd, const uint4 *bop, int lds_units, float *apart);
hipError_t launch_adj_reduce(const ConvLaunch &L, int nrows_out, const int32_t *row_ptr,
                             const int64_t *entry_off, const float *apart, int accumulate,
                             float *g);

// Per replica column r: out[2r] = sum_i (y - ref)^2, out[2r+1] = sum_i ref^2
// (FP64), for y and ref [N][R].
hipError_t launch_col_err(const float *y, const float *ref, int N, int R, double *out,
                          hipStream_t s);

// Static scratch of the allocation-free DIS entry point: kStaticScratchBytes
// of device memory per GPU (a file-scope __device__ array).  resolve() looks
// up the array's device address on ``device`` (which must be current) once;
// static_scratch() returns it (nullptr before resolve).
constexpr size_t kStaticScratchBytes = 4u << 20;
constexpr int kMaxDevices = 64;
hipError_t static_scratch_resolve(int device);
void *static_scratch(int device);

// Flattened form of Table 3 (flat_kernels.hip).  Active flavour pairs of
// the luminosity, a * 64 + b, in row-major (a, b) order.
constexpr int kFlatMaxPairs = 1024;
struct FlatPairs {
  int32_t n;
  int16_t ab[kFlatMaxPairs];
};
// Launch shape of out[N][R] = FK[N][K] L[K][R]: the matrix-core kernel
// (128 x 128 tiles) or the streaming kernel (nb rows x cw*vec columns), K split
// into ks chunks of kchunk (partial sums in a workspace when ks > 1).
struct FlatPlan {
  bool mfma = false;
  int nb = 8, cw = 1, vec = 1, ks = 1;
  int64_t gx = 1, gy = 1, kchunk = 0;
  uint64_t work_bytes = 0;
};
FlatPlan flat_plan(int64_t N, int64_t K, int64_t R, int ncu);
hipError_t launch_lumi(const FlatPairs &pairs, int nx, int R, const float *pdf, float *lum,
                       hipStream_t s);
hipError_t launch_flat(const FlatPlan &p, int64_t N, int64_t K, int64_t R, const float *fk,
                       const float *lum, float *out, float *work, hipStream_t s);

// Network PDF (mlp_kernels.hip): one network per replica on the x-grid;
// d_xin = [2][X] (x, ln x), d_pre = [F][X] (x^alpha (1-x)^beta).
constexpr int kMlpMaxNx = 256;          // grid points (one thread each)
constexpr size_t kMlpMaxLds = 65536;    // LDS of one replica's workgroup
struct MlpDev {
  int F = 0, X = 0, h1 = 0, h2 = 0;
  const float *d_xin = nullptr, *d_pre = nullptr;
};
int mlp_nparams(int F, int h1, int h2);
size_t mlp_lds_bytes(int F, int X, int h1, int h2, bool backward);
hipError_t launch_mlp_forward(const MlpDev &m, const float *params, int R, float *pdf, hipStream_t s);
hipError_t launch_mlp_backward(const MlpDev &m, const float *params, const float *gpdf, int R,
                               float *gparams, hipStream_t s);
hipError_t launch_sgd(float *params, const float *grad, int64_t n, float lr, hipStream_t s);

// chi2 (chi2_kernels.hip)
hipError_t launch_cholesky(int nblocks, const int32_t *d_n, const int64_t *d_off, double *d_a,
                           double *d_linv, int32_t *d_flag, int maxn, hipStream_t s);
// Per-call chi2 work of a covariance: row tiles (32 rows of a block), and
// the split products: entries {row tile, first k tile, end k tile, slot},
// those of row tile rt at [ptr[rt], ptr[rt + 1]).
constexpr int kChi2Split = 4;  // k tiles per entry of the split products (at least)
struct Chi2Plan {
  int nrt = 0, nlw = 0, nuw = 0;
  const int32_t *d_rt_block = nullptr, *d_rt_row = nullptr, *d_n = nullptr, *d_roff = nullptr;
  const int64_t *d_off = nullptr;
  const int4 *d_lw = nullptr, *d_uw = nullptr;
  const int32_t *d_lptr = nullptr, *d_uptr = nullptr;
  double *d_spart = nullptr;  // [max(nlw, nuw)][32][kRpMax]
  double *d_y = nullptr;      // [ntot][kRpMax]
  double *d_part = nullptr;   // [nrt][kRpMax]
};
hipError_t launch_chi2(const Chi2Plan &P, const double *d_linv, const float *sigma,
                       const double *data, int R, int c0, int ncols, double *chi2, float *dchi2,
                       hipStream_t s);

}  // namespace fk
