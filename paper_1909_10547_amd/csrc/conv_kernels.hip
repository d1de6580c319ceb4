// HIP kernels of the FK-table convolution for gfx950 (MI355X).
//
// The hot loop of every kernel is a 16 x 16*NT MFMA tile per wave64:
//   rows    = 16 datapoints (forward, hadronic adjoint) or 16 (flavour, x)
//             rows of a transposed DIS table (DIS adjoint),
//   columns = PDF replicas,
//   k       = the concatenated (flavour, x) index of one group of partner
//             flavours (FK rows are split into groups so that the group's
//             B operand fits in LDS).
// The FK operand streams from HBM once, 16 bytes per lane per k-step, in
// the fragment order written by the host packer (fully coalesced 1 KiB per
// wave per k-step); the B operand is staged in LDS by the workgroup.
//
//  DIS (Section 3, linear convolution):   T[i,r] = s_i sum_k FKhat[i,k] f[k,r]
//  hadronic (Eq. (1)):  sigma[i,r] = (s_i/2) sum_p f[p,r] sum_q Shat_i[p,q] f[q,r]
//    with S_i = FK_i + FK_i^T the symmetric part of the table (Eq. (1) only
//    sees it); H = Shat f is the MFMA product and the dot with f[p,r] is the
//    fused epilogue, so H never leaves registers.
//  adjoints (Table 1, "Gradient"):  DIS g = sum_i FK_i gbar_i,
//    hadronic g[p,r] = sum_i gbar[i,r] s_i (Shat_i f)[p,r]  -- the same MFMA
//    product as the forward pass with a different epilogue.
// Where a row's sum is split over workgroups, the parts go to slots that
// are reduced in a fixed order (the DIS stream kernel writes whole rows
// itself), so results are bitwise reproducible and independent of batch
// composition.
#include <algorithm>
#include <mutex>

#include "fk_internal.h"

namespace fk {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// MFMA per 16-byte unit.  Lane l supplies unit (4t + l/16) of its row for A
// and of its column for B; whatever order the hardware assigns to the k
// elements inside a lane, A and B use the same one, so the contraction is
// exact.  Output layout (16x16 f32): lane l holds rows 4*(l/16)+q, q=0..3,
// of column l%16.
// ---------------------------------------------------------------------------
template <int DT>
struct Mma;

template <>
struct Mma<FK_BF16> {
  static constexpr int E = 8;
  static __device__ __forceinline__ void run(u32x4 a, u32x4 b, f32x4 &c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
  // c = a * b (the accumulator operand is the constant zero)
  static __device__ __forceinline__ void first(u32x4 a, u32x4 b, f32x4 &c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b),
                                                f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  }
};

template <>
struct Mma<FK_F32> {
  static constexpr int E = 4;
  static __device__ __forceinline__ void run(u32x4 a, u32x4 b, f32x4 &c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
  }
  static __device__ __forceinline__ void first(u32x4 a, u32x4 b, f32x4 &c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x),
                                             f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
  }
};

template <>
struct Mma<FK_FP8E4M3> {
  static constexpr int E = 16;
  static __device__ __forceinline__ void run(u32x4 a, u32x4 b, f32x4 &c) {
    const long a0 = (long)(((unsigned long)a.y << 32) | a.x);
    const long a1 = (long)(((unsigned long)a.w << 32) | a.z);
    const long b0 = (long)(((unsigned long)b.y << 32) | b.x);
    const long b1 = (long)(((unsigned long)b.w << 32) | b.z);
    c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void first(u32x4 a, u32x4 b, f32x4 &c) {
    c = f32x4{0.f, 0.f, 0.f, 0.f};
    run(a, b, c);
  }
};

// Table pointers come from descriptors in memory, so the compiler cannot
// infer their address space and would emit flat loads, which count against
// the LDS wait counter as well: every LDS read of the B operand would then
// wait for the in-flight HBM prefetch.  The tables live in global memory.
typedef const __attribute__((address_space(1))) u32x4 *gu32x4_ptr;
// Buffer descriptors (raw, stride 0): the fourth word of a gfx9-family
// descriptor for untyped 32-bit accesses, and the load cache policy
// "non-temporal" (the table streams once).
constexpr int kBufferRsrcWord3 = 0x00020000;
constexpr int kLoadNT = 2;
__device__ __forceinline__ gu32x4_ptr as_global(const void *p) { return (gu32x4_ptr)p; }

// A operand of one tile: T k-steps of the row block stored unit-major
// (unit u of row rho at base[u*nv + rho]); rows >= nv, units >= KE and
// k-steps >= T read the zero page ``zp`` (64 zero units, always mapped).
// Every tile thus issues exactly kTMax loads, so the compiler can wait for
// one tile precisely while the next tile's loads stay in flight.
__device__ __forceinline__ void load_a(u32x4 (&a)[kTMax], const u32x4 *base_generic, int nv,
                                       int KE, const u32x4 *zp_generic) {
  const gu32x4_ptr base = as_global(base_generic);
  const gu32x4_ptr zp = as_global(zp_generic);
  const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
#pragma unroll
  for (int t = 0; t < kTMax; ++t) {
    const int u = 4 * t + g;
    const bool ok = row < nv && u < KE;
    a[t] = __builtin_nontemporal_load(ok ? base + (size_t)u * nv + row : zp + lane);
  }
}

// acc[j] += A (16 x 4T units) * B (4T units x 16 columns of tile j); B in
// LDS as [unit][RP].  The B fragments of k-step t+1 are read while the
// MFMAs of k-step t issue; the scheduling barrier keeps the compiler from
// hoisting every LDS read of the tile (which would cost NT*4*T registers).
template <int DT, int NT>
__device__ __forceinline__ void mma_tile(const u32x4 (&a)[kTMax], int T,
                                         const u32x4 *__restrict__ lb, f32x4 (&acc)[NT]) {
  constexpr int RP = 16 * NT;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const u32x4 *bp = lb + g * RP + c;
#pragma unroll
  for (int t = 0; t < kTMax; ++t) {
    if (t < T) {
      u32x4 b[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j) b[j] = bp[(4 * t) * RP + 16 * j];
#pragma unroll
      for (int j = 0; j < NT; ++j) Mma<DT>::run(a[t], b[j], acc[j]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int NT>
__device__ __forceinline__ void zero(f32x4 (&v)[NT]) {
#pragma unroll
  for (int j = 0; j < NT; ++j) v[j] = f32x4{0.f, 0.f, 0.f, 0.f};
}

__device__ __forceinline__ void copy_b(u32x4 *__restrict__ lds, const u32x4 *__restrict__ src,
                                       int n) {
  for (int i = threadIdx.x; i < n; i += kThreads) lds[i] = src[i];
}

// ---------------------------------------------------------------------------
// Rounding of the B operand (round to nearest, ties to even)
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned f32_to_bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// OCP e4m3fn: 1-4-3, bias 7, max 448, no infinities; saturating.
__device__ __forceinline__ unsigned f32_to_e4m3_bits(float x) {
  const unsigned sign = (__float_as_uint(x) >> 24) & 0x80u;
  float ax = fabsf(x);
  if (!(ax == ax)) return 0x7fu;  // NaN
  if (ax >= 448.f) return sign | 0x7eu;
  if (ax < 0.015625f) {  // below 2^-6: subnormal grid of 2^-9
    const unsigned q = (unsigned)rintf(ax * 512.f);  // 0..8, 8 encodes 2^-6
    return sign | q;
  }
  int e = ((__float_as_uint(ax) >> 23) & 0xff) - 127;  // ax in [2^e, 2^(e+1))
  float q = rintf(ldexpf(ax, 3 - e));                   // 8..16
  if (q >= 16.f) {
    q = 8.f;
    ++e;
  }
  unsigned code = ((unsigned)(e + 7) << 3) | ((unsigned)q - 8u);
  return sign | (code > 0x7eu ? 0x7eu : code);
}

template <int DT>
__device__ __forceinline__ u32x4 pack_unit(const float *v);

template <>
__device__ __forceinline__ u32x4 pack_unit<FK_F32>(const float *v) {
  return u32x4{__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
               __float_as_uint(v[3])};
}
template <>
__device__ __forceinline__ u32x4 pack_unit<FK_BF16>(const float *v) {
  u32x4 r;
  r.x = f32_to_bf16_bits(v[0]) | (f32_to_bf16_bits(v[1]) << 16);
  r.y = f32_to_bf16_bits(v[2]) | (f32_to_bf16_bits(v[3]) << 16);
  r.z = f32_to_bf16_bits(v[4]) | (f32_to_bf16_bits(v[5]) << 16);
  r.w = f32_to_bf16_bits(v[6]) | (f32_to_bf16_bits(v[7]) << 16);
  return r;
}
template <>
__device__ __forceinline__ u32x4 pack_unit<FK_FP8E4M3>(const float *v) {
  unsigned w[4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
    w[m] = f32_to_e4m3_bits(v[4 * m]) | (f32_to_e4m3_bits(v[4 * m + 1]) << 8) |
           (f32_to_e4m3_bits(v[4 * m + 2]) << 16) | (f32_to_e4m3_bits(v[4 * m + 3]) << 24);
  return u32x4{w[0], w[1], w[2], w[3]};
}

// ---------------------------------------------------------------------------
// B-operand staging: for every group descriptor, the [KEpad][RP] unit array
// of B[k, n] = src[row(k)][c0 + n] (times s_row for the adjoint weights),
// rounded to the storage format, zero for k >= K or n >= ncols.
// ---------------------------------------------------------------------------
template <int DT>
__global__ void __launch_bounds__(kThreads)
    stage_b_kernel(const GroupDesc *__restrict__ gd, const int32_t *__restrict__ rowtab, int ngd,
                   const float *__restrict__ pdf, const float *__restrict__ gout,
                   const float *__restrict__ scale_all, int R, int c0, int ncols, int RP,
                   u32x4 *__restrict__ bop, int *counter, float *__restrict__ fstage, int nx,
                   const int32_t *__restrict__ wrow, float *__restrict__ wstage, int nwpair) {
  constexpr int E = Mma<DT>::E;
  // the forward kernel that follows on the stream takes items from *counter
  if (counter && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *counter = 0;
  // grid: x = chunk of kThreads units (or floats), y = descriptor
  const int idx = blockIdx.x * kThreads + threadIdx.x;
  if ((int)blockIdx.y >= ngd && wstage) {
    // rows past the descriptors: the adjoint weights gbar * s of each block
    // pair, column by column [pair][RP][kAdjWRow], zero for columns >=
    // ncols, padding rows and the pad of a column
    const size_t i = (size_t)(blockIdx.y - ngd) * gridDim.x * kThreads + idx;
    if (i >= (size_t)nwpair * RP * kAdjWRow) return;
    const int q = (int)(i % kAdjWRow);
    const size_t pn = i / kAdjWRow;
    const int n = (int)(pn % RP), P = (int)(pn / RP);
    const int r = q < 32 ? wrow[32 * P + q] : -1;
    wstage[i] = r >= 0 && n < ncols ? gout[(size_t)r * R + c0 + n] * scale_all[r] : 0.f;
    return;
  }
  if ((int)blockIdx.y >= ngd) {
    // rows past the descriptors: FP32 PDF rows of flavour a for the
    // epilogue of the stream kernel, [alpha][RP], zero for columns >= ncols
    const int a = blockIdx.y - ngd;
    if (idx >= nx * RP) return;
    const int al = idx / RP, n = idx - al * RP;
    fstage[(size_t)a * nx * RP + idx] = n < ncols ? pdf[((size_t)a * nx + al) * R + c0 + n] : 0.f;
    return;
  }
  const GroupDesc *G = gd + blockIdx.y;
  const int KEpad = ((G->KE + 3) >> 2) << 2;
  if (idx >= KEpad * RP) return;
  const int src_kind = G->src;
  const float *src = src_kind == 0 ? pdf : gout;
  const int u = idx / RP, n = idx - u * RP;
  // the unit's E source rows (-1 past the contraction length), read as
  // 16-byte vectors: every thread of a unit reads the same ones
  int row[E];
  const int32_t *rp = rowtab + G->row_off + (size_t)u * E;
#pragma unroll
  for (int q = 0; q < E / 4; ++q) {
    const int4 r4 = *(const int4 *)(rp + 4 * q);
    row[4 * q] = r4.x;
    row[4 * q + 1] = r4.y;
    row[4 * q + 2] = r4.z;
    row[4 * q + 3] = r4.w;
  }
  float v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    float x = 0.f;
    if (row[e] >= 0 && n < ncols) {
      x = src[(size_t)row[e] * R + c0 + n];
      if (src_kind == 1) x *= scale_all[row[e]];
    }
    v[e] = x;
  }
  bop[G->bop_off + idx] = pack_unit<DT>(v);
}

// f[a][alpha][c0 + 16j + lane%16] for the epilogue; columns >= ncols (and
// a row beyond the grid, row == nullptr) read the zero page.
template <int NT>
__device__ __forceinline__ void load_f(float (&f)[NT], const float *row, int ncols,
                                       const u32x4 *zp) {
  const int c = threadIdx.x & 15;
  const float *z = (const float *)zp;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int col = 16 * j + c;
    f[j] = *((row && col < ncols) ? row + col : z + c);
  }
}

// Workgroup barrier that orders LDS only: global loads in flight (the next
// tiles of the FK stream) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Two tiles at the same x index alpha: rows = datapoints of two consecutive
// 16-datapoint blocks (the second may be absent).  Both tiles multiply the
// same B fragments, which halves the LDS traffic per byte of table.
struct TilePair {
  const u32x4 *p0, *p1;
  int nv0, nv1, KE;
  const float *frow;  // f[a][alpha][c0..], nullptr for an empty pair
};

// k-step t of ``n`` into a0[t], a1[t]; lanes outside a tile read the zero page
__device__ __forceinline__ void refill(u32x4 (&a0)[kTMax], u32x4 (&a1)[kTMax], int t,
                                       const TilePair &n, const u32x4 *zp_generic) {
  const gu32x4_ptr zp = as_global(zp_generic);
  const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
  const int u = 4 * t + g;
  const bool ok0 = row < n.nv0 && u < n.KE;
  const bool ok1 = row < n.nv1 && u < n.KE;
  a0[t] = __builtin_nontemporal_load(ok0 ? as_global(n.p0) + (size_t)u * n.nv0 + row : zp + lane);
  a1[t] = __builtin_nontemporal_load(ok1 ? as_global(n.p1) + (size_t)u * n.nv1 + row : zp + lane);
}

// MFMAs of the current pair (TT k-steps) with the next pair's loads issued
// into each k-step's registers as soon as that k-step has been multiplied;
// k-steps TT..kTMax-1 of the next pair are loaded after the loop.  Every pair
// issues the same number of loads, so the waits are exact.
template <int DT, int NT, int TT>
__device__ __forceinline__ void pair_mma(u32x4 (&a0)[kTMax], u32x4 (&a1)[kTMax],
                                         const u32x4 *__restrict__ lb, f32x4 (&acc0)[NT],
                                         f32x4 (&acc1)[NT], const TilePair &nxt,
                                         float (&fn)[NT], int ncols, const u32x4 *zp) {
  constexpr int RP = 16 * NT;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const u32x4 *bp = lb + g * RP + c;
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    u32x4 b[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) b[j] = bp[4 * t * RP + 16 * j];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      Mma<DT>::run(a0[t], b[j], acc0[j]);
      Mma<DT>::run(a1[t], b[j], acc1[j]);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (t == 0) load_f<NT>(fn, nxt.frow, ncols, zp);
    refill(a0, a1, t, nxt, zp);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int t = TT; t < kTMax; ++t) refill(a0, a1, t, nxt, zp);
}

// ---------------------------------------------------------------------------
// Hadronic forward.  Persistent workgroups take items (two 16-datapoint
// blocks x a run of row groups) from a counter; wave w owns the x indices
// alpha = w (mod 4) of both blocks and keeps its running dot products
// sigma partial sums for the two blocks in registers.
// ---------------------------------------------------------------------------
template <int DT, int NT>
__global__ void __launch_bounds__(kThreads)
    had_fwd_kernel(const FwdItem *__restrict__ items, int nitems, const SegRef *__restrict__ segs,
                   const GroupDesc *__restrict__ gd, const u32x4 *__restrict__ bop,
                   const float *__restrict__ pdf, int R, int c0, int ncols, int nx,
                   float *__restrict__ part, const u32x4 *zp, int *counter) {
  constexpr int RP = 16 * NT;
  constexpr int S = kWaves;
  extern __shared__ u32x4 lds[];
  __shared__ int s_item;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  u32x4 a0[kTMax], a1[kTMax];
  float f[NT], fn[NT];
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    lds_barrier();
    const int item = s_item;
    if (item >= nitems) break;
    const FwdItem it = items[item];
    const int bl0 = it.block0;
    const int nv0 = min(16, it.ndata - 16 * bl0);
    const int nv1 = it.nblk > 1 ? min(16, it.ndata - 16 * (bl0 + 1)) : 0;
    auto pair_at = [&](int s, int al) {
      TilePair p{zp, zp, 0, 0, 1, nullptr};
      if (s < it.seg1 && al < nx) {
        const SegRef sr = segs[s];
        const u32x4 *base = (const u32x4 *)sr.base;
        p.KE = sr.KE;
        p.nv0 = nv0;
        p.nv1 = nv1;
        // [pair][alpha][block of the pair][unit][row] (see the packer)
        p.p0 = base + ((size_t)bl0 * nx * 16 + (size_t)al * (nv0 + nv1)) * sr.KE;
        p.p1 = nv1 ? p.p0 + (size_t)nv0 * sr.KE : zp;
        p.frow = pdf + ((size_t)gd[sr.gdesc].a * nx + al) * R + c0;
      }
      return p;
    };
    f32x4 sacc0[NT], sacc1[NT];
    zero(sacc0);
    zero(sacc1);
    {  // first pair of the item
      const TilePair p = pair_at(it.seg0, w);
#pragma unroll
      for (int t = 0; t < kTMax; ++t) refill(a0, a1, t, p, zp);
      load_f<NT>(f, p.frow, ncols, zp);
    }
    for (int s = it.seg0; s < it.seg1; ++s) {
      const SegRef sr = segs[s];
      const int T = (sr.KE + 3) >> 2;
      lds_barrier();
      copy_b(lds, bop + gd[sr.gdesc].bop_off, 4 * T * RP);
      lds_barrier();
      for (int al = w; al < nx; al += S) {
        const int aln = al + S < nx ? al + S : w;
        const TilePair nxt = pair_at(al + S < nx ? s : s + 1, aln);
        f32x4 acc0[NT], acc1[NT];
        zero(acc0);
        zero(acc1);
        switch (T) {
          case 1: pair_mma<DT, NT, 1>(a0, a1, lds, acc0, acc1, nxt, fn, ncols, zp); break;
          case 2: pair_mma<DT, NT, 2>(a0, a1, lds, acc0, acc1, nxt, fn, ncols, zp); break;
          case 3: pair_mma<DT, NT, 3>(a0, a1, lds, acc0, acc1, nxt, fn, ncols, zp); break;
          case 4: pair_mma<DT, NT, 4>(a0, a1, lds, acc0, acc1, nxt, fn, ncols, zp); break;
          case 5: pair_mma<DT, NT, 5>(a0, a1, lds, acc0, acc1, nxt, fn, ncols, zp); break;
          case 6: pair_mma<DT, NT, 6>(a0, a1, lds, acc0, acc1, nxt, fn, ncols, zp); break;
          case 7: pair_mma<DT, NT, 7>(a0, a1, lds, acc0, acc1, nxt, fn, ncols, zp); break;
          default: pair_mma<DT, NT, 8>(a0, a1, lds, acc0, acc1, nxt, fn, ncols, zp); break;
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          sacc0[j] += acc0[j] * f[j];
          sacc1[j] += acc1[j] * f[j];
          f[j] = fn[j];
        }
      }
    }
    // combine the waves' partial sums in a fixed order, one slot per block
    lds_barrier();
    float *red = (float *)lds;  // [block][wave][16][RP]
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        red[((0 * S + w) * 16 + 4 * g + q) * RP + 16 * j + c] = sacc0[j][q];
        red[((1 * S + w) * 16 + 4 * g + q) * RP + 16 * j + c] = sacc1[j][q];
      }
    lds_barrier();
    for (int b = 0; b < it.nblk; ++b) {
      const float *rb = red + (size_t)b * S * 16 * RP;
      float *dst = part + (size_t)(it.slot0 + b) * 16 * kRpMax;
      for (int i = threadIdx.x; i < 16 * RP; i += kThreads) {
        const int row = i / RP, col = i - row * RP;
        dst[row * kRpMax + col] =
            ((rb[i] + rb[16 * RP + i]) + rb[32 * RP + i]) + rb[48 * RP + i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Stream kernel (hadronic forward and adjoint).  Each workgroup walks a
// static list of records: forward, one group of an item (a block pair and a
// run of groups); adjoint, one block pair of an item (an adjoint group and a
// run of block pairs).  The waves split alpha (alpha = w mod S).  Seen from
// one wave, the FK tiles of its (record, alpha) jobs form one flat stream of
// k-steps (T per job), and a ring of W k-steps of both tiles of the pair
// stays in flight in registers, so the bytes in flight do not depend on the
// group size.  Every k-step issues exactly two loads, which keeps the
// compiler's waits on the ring exact.
//
// The B operand and the epilogue rows of each record (forward: the FP32 PDF
// rows of its flavour; adjoint: the weights of its 32 datapoints) go to one
// of two LDS buffers by LDS-DMA.  The copies of record r+1 are issued right
// after the barrier that starts record r, which released the buffer of
// record r-1; at the change to r+1 each wave waits for its own copies (they
// were issued before all the ring loads of record r, at least 2W of them,
// since every record lasts at least W k-steps per wave: the host checks
// this) and a workgroup barrier publishes them.  Forward: at the end of an
// item the waves' partial sums are combined in a fixed order in the buffer
// of the record just finished and written to the item's slots.  Adjoint:
// each wave keeps the gradient rows of its alpha in registers and writes
// them to the item's slot at its end.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt is six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// One LDS-DMA instruction: lane l copies 16 bytes from ``src`` (its own
// address) to LDS ``dst`` + 16 l (``dst`` uniform, set in M0).  Written as
// inline assembly so that the compiler does not treat it as a pending write
// to all of LDS: it would then wait for every load in flight (vmcnt(0))
// before each LDS read of the other buffer.  The copies are waited for
// explicitly (wait_vmcnt); the compiler's own waits on the ring only grow
// stricter from loads it does not count.
__device__ __forceinline__ void dma16(gu32x4_ptr src, u32x4 *dst) {
  const unsigned l = (unsigned)(uintptr_t)(__attribute__((address_space(3))) void *)dst;
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
               :
               : "s"(__builtin_amdgcn_readfirstlane(l)), "v"(src)
               : "memory", "m0");
}

// Copy ``units`` 16-byte units from global ``src`` to LDS ``dst``:
// instruction k moves units [64k, 64k+64); wave w issues instructions w,
// w+4, ...  Lanes past the end read the zero page and write inside the last
// KiB of the copy (buffers are whole KiB).
template <int S>
__device__ __forceinline__ void dma_copy(u32x4 *dst, const u32x4 *src, int units,
                                         const u32x4 *zp, int w, int lane) {
  const int n = (units + 63) >> 6;
  for (int k = w; k < n; k += S) {
    const int u = 64 * k + lane;
    dma16(u < units ? as_global(src) + u : as_global(zp) + lane, dst + 64 * k);
  }
}

template <int DT, int NT, int W, int S, int MODE>
__global__ void __launch_bounds__(64 * S, 1)
    had_stream_kernel(const StreamSeg *__restrict__ recs, const int32_t *__restrict__ wg_ptr,
                      const u32x4 *__restrict__ bop, const float *__restrict__ fstage, int nx,
                      int bufsz, float *__restrict__ part, const u32x4 *zp) {
  constexpr int RP = 16 * NT;
  constexpr int NTHR = 64 * S;
  constexpr bool ADJ = MODE == kStreamAdj;
  extern __shared__ u32x4 lds[];
  // the wave index is uniform: say so, so that every cursor below lives in
  // scalar registers and every branch on it is a scalar branch
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int r_begin = wg_ptr[blockIdx.x], r_end = wg_ptr[blockIdx.x + 1];
  if (r_begin >= r_end) return;

  u32x4 a0[W], a1[W];
  f32x4 acc0[NT], acc1[NT], sacc0[NT], sacc1[NT];
  zero(acc0);
  zero(acc1);
  zero(sacc0);
  zero(sacc1);
  // adjoint: the gradient rows of the wave's x indices alpha = w + S k; lane
  // (g, c) keeps k = g (gr0) and k = g + 4 (gr1)
  // (vectors, so that they stay in registers whatever the inliner does)
  typedef float f32x8 __attribute__((ext_vector_type(8)));
  static_assert(NT <= 8, "eight column tiles at most");
  f32x8 gr0 = f32x8(0.f), gr1 = f32x8(0.f);

  // B operand of record ``q`` and its epilogue rows into buffer ``par``:
  // forward, the FP32 PDF rows of its flavour; adjoint, the weights of its
  // two blocks
  auto stage = [&](const StreamSeg &q, int par) {
    u32x4 *buf = lds + par * bufsz;
    const int ub = 4 * q.T * RP;
    dma_copy<S>(buf, bop + q.bop_off, ub, zp, w, lane);
    if (ADJ)
      dma_copy<S>(buf + ub, (const u32x4 *)(fstage + (size_t)q.flav * RP * kAdjWRow),
                  RP * kAdjWRow / 4, zp, w, lane);
    else
      dma_copy<S>(buf + ub, (const u32x4 *)(fstage + (size_t)q.flav * nx * RP), nx * RP / 4, zp,
                  w, lane);
  };

  // refill cursor: record rr, job alpha r_al, k-step r_t.  The two tiles
  // of the current job are read through buffer descriptors whose size is the
  // tile, so the hardware returns zeros for units past the row's end (u >=
  // KE); lanes whose row is absent (row >= nv) get an offset beyond any
  // tile; past the end of the list the descriptors are empty.  The lane's
  // offset within a k-step is fixed per record; the k-step adds a uniform
  // offset.
  int rr = r_begin, r_al = w, r_t = 0;
  bool r_done = false;
  StreamSeg Rq = recs[rr];
  // forward copy: the two tiles of a pair alternate at every alpha (see the
  // packer); adjoint copy: each block's tiles follow one another
  auto stride0 = [](const StreamSeg &q) { return (size_t)(ADJ ? q.nv0 : q.nv0 + q.nv1) * q.KE; };
  auto stride1 = [](const StreamSeg &q) { return (size_t)(ADJ ? q.nv1 : q.nv0 + q.nv1) * q.KE; };
  constexpr unsigned kNoRow = 0x80000000u;  // beyond every tile (<= 8 KiB)
  __amdgpu_buffer_rsrc_t rs0, rs1;
  unsigned vo0 = 0, vo1 = 0, ko0 = 0, ko1 = 0;
  auto set_tiles = [&]() {
    const u32x4 *p0 = (const u32x4 *)Rq.a0 + r_al * stride0(Rq);
    const u32x4 *p1 = Rq.a1 ? (const u32x4 *)Rq.a1 + r_al * stride1(Rq) : zp;
    rs0 = __builtin_amdgcn_make_buffer_rsrc((void *)p0, (short)0, r_done ? 0 : Rq.KE * Rq.nv0 * 16,
                                            kBufferRsrcWord3);
    rs1 = __builtin_amdgcn_make_buffer_rsrc((void *)p1, (short)0, r_done ? 0 : Rq.KE * Rq.nv1 * 16,
                                            kBufferRsrcWord3);
    ko0 = ko1 = 0;
  };
  auto set_lanes = [&]() {
    vo0 = c < Rq.nv0 ? (unsigned)(g * Rq.nv0 + c) * 16u : kNoRow;
    vo1 = c < Rq.nv1 ? (unsigned)(g * Rq.nv1 + c) * 16u : kNoRow;
  };
  set_tiles();
  set_lanes();
  // Two loads per call on every path (past the end of the list, of empty
  // descriptors); the cursor advance has no loads.
  auto refill = [&](u32x4 &x0, u32x4 &x1) {
    x0 = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs0, vo0 + ko0, 0, kLoadNT));
    x1 = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs1, vo1 + ko1, 0, kLoadNT));
    if (!r_done) {
      ko0 += 64u * Rq.nv0;
      ko1 += 64u * Rq.nv1;
      if (++r_t == Rq.T) {
        r_t = 0;
        r_al += S;
        if (r_al >= nx) {
          r_al = w;
          if (++rr == r_end) {
            r_done = true;
          } else {
            Rq = recs[rr];
            set_lanes();
          }
        }
        set_tiles();
      }
    }
  };

  // The waves' sums of the item, combined in a fixed order: with eight
  // waves, wave w + 4 first adds its sums into wave w's (w < 4); then the
  // four remaining sums are added in wave order.
  // Adjoint: the item's gradient rows go straight from the registers to its
  // slot [x][kRpMax]; no other wave holds the same x index.
  auto flush_adj = [&](const StreamSeg &q) {
    float *dst = part + (size_t)q.slot * nx * kRpMax + 16 * 0 + c;
    const int al0 = w + S * g, al1 = w + S * (g + 4);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      if (al0 < nx) dst[(size_t)al0 * kRpMax + 16 * j] = gr0[j];
      if (al1 < nx) dst[(size_t)al1 * kRpMax + 16 * j] = gr1[j];
    }
    gr0 = f32x8(0.f);
    gr1 = f32x8(0.f);
  };
  auto flush = [&](const StreamSeg &q, int par) {
    float *red = (float *)(lds + par * bufsz);  // [block][4][16][RP]
    auto put = [&](int slot) {
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          red[((0 * 4 + slot) * 16 + 4 * g + e) * RP + 16 * j + c] = sacc0[j][e];
          red[((1 * 4 + slot) * 16 + 4 * g + e) * RP + 16 * j + c] = sacc1[j][e];
        }
    };
    lds_barrier();
    if (S == 8) {
      if (w >= 4) put(w - 4);
      lds_barrier();
      if (w < 4) {
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            sacc0[j][e] += red[((0 * 4 + w) * 16 + 4 * g + e) * RP + 16 * j + c];
            sacc1[j][e] += red[((1 * 4 + w) * 16 + 4 * g + e) * RP + 16 * j + c];
          }
      }
      lds_barrier();
    }
    if (w < 4) put(w);
    lds_barrier();
    // the item's slots, through descriptors over them: a fixed number of
    // stores on every path (elements past the tile and the slot of an
    // absent second block are dropped by the descriptors), so the
    // compiler's waits on the ring do not have to drain it here
    constexpr int kPer = (16 * RP + NTHR - 1) / NTHR;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const float *rb = red + (size_t)b * 4 * 16 * RP;
      const __amdgpu_buffer_rsrc_t rsd = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(part + (size_t)(q.slot + b) * 16 * kRpMax), (short)0,
          b == 0 || q.nv1 > 0 ? 16 * kRpMax * 4 : 0, kBufferRsrcWord3);
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int i = threadIdx.x + k * NTHR;
        const int ii = i < 16 * RP ? i : 0;
        const int rw = ii / RP, col = ii - rw * RP;
        const float v = ((rb[ii] + rb[16 * RP + ii]) + rb[32 * RP + ii]) + rb[48 * RP + ii];
        const unsigned off = i < 16 * RP ? (unsigned)(rw * kRpMax + col) * 4u : 0x80000000u;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rsd, off, 0, 0);
      }
    }
    lds_barrier();
    zero(sacc0);
    zero(sacc1);
  };

  // consume cursor: record cr, job alpha c_al, k-step c_t, buffer cpar.
  // The B fragments of a k-step are read right after the MFMAs of the one
  // before (same registers), so their LDS latency overlaps the epilogue, the
  // cursor work and the refill.
  int cr = r_begin, c_al = w, c_t = 0, cpar = 0, c_k = 0;
  StreamSeg Cq = Rq;
  bool done = false;
  u32x4 b[NT];
  auto read_b = [&]() {
    const u32x4 *bp = lds + cpar * bufsz + (4 * c_t + g) * RP + c;
#pragma unroll
    for (int j = 0; j < NT; ++j) b[j] = bp[16 * j];
  };

  auto consume = [&](const u32x4 &x0, const u32x4 &x1) {
    if (done) return;
    // the first k-step of a job starts the accumulators from zero
    if (c_t == 0) {
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        Mma<DT>::first(x0, b[j], acc0[j]);
        Mma<DT>::first(x1, b[j], acc1[j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        Mma<DT>::run(x0, b[j], acc0[j]);
        Mma<DT>::run(x1, b[j], acc1[j]);
      }
    }
    const bool job_end = ++c_t == Cq.T;
    const bool rec_end = job_end && c_al + S >= nx;
    if (job_end) c_t = 0;
    // the next k-step's B, unless the group changes (its buffer is then
    // published by the barrier below)
    if (!rec_end) read_b();
    if (job_end) {
      if (ADJ) {
        // sum over the 16 rows of each tile of acc times the weights (the
        // lane's four rows are one 16-byte read of a weight column; the
        // tile of an absent second block is skipped).  Each step runs over
        // all column tiles before the next one starts, so the weight reads
        // and each round of cross-lane adds are issued together and wait
        // once (per tile they would form one chain of LDS round trips).
        const float *wt = (const float *)(lds + cpar * bufsz + 4 * Cq.T * RP) + c * kAdjWRow + 4 * g;
        float v[NT];
        if (Cq.nv1 > 0) {
          f32x4 w0[NT], w1[NT];
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            w0[j] = *(const f32x4 *)(wt + 16 * j * kAdjWRow);
            w1[j] = *(const f32x4 *)(wt + 16 * j * kAdjWRow + 16);
          }
#pragma unroll
          for (int j = 0; j < NT; ++j)
            v[j] = (((acc0[j][0] * w0[j][0] + acc0[j][1] * w0[j][1]) + acc0[j][2] * w0[j][2]) +
                    acc0[j][3] * w0[j][3]) +
                   (((acc1[j][0] * w1[j][0] + acc1[j][1] * w1[j][1]) + acc1[j][2] * w1[j][2]) +
                    acc1[j][3] * w1[j][3]);
        } else {
          f32x4 w0[NT];
#pragma unroll
          for (int j = 0; j < NT; ++j) w0[j] = *(const f32x4 *)(wt + 16 * j * kAdjWRow);
#pragma unroll
          for (int j = 0; j < NT; ++j)
            v[j] = ((acc0[j][0] * w0[j][0] + acc0[j][1] * w0[j][1]) + acc0[j][2] * w0[j][2]) +
                   acc0[j][3] * w0[j][3];
        }
        float u[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) u[j] = __shfl_xor(v[j], 16);
#pragma unroll
        for (int j = 0; j < NT; ++j) v[j] += u[j];
#pragma unroll
        for (int j = 0; j < NT; ++j) u[j] = __shfl_xor(v[j], 32);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          v[j] += u[j];
          // branch-free: both rows are updated, one of them by zero
          gr0[j] += g == c_k ? v[j] : 0.f;
          gr1[j] += g == c_k - 4 ? v[j] : 0.f;
        }
      } else {
        const float *fl = (const float *)(lds + cpar * bufsz + 4 * Cq.T * RP) + c_al * RP + c;
        float fv[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) fv[j] = fl[16 * j];
        // one column tile at a time keeps few accumulators in flight
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          sacc0[j] += acc0[j] * fv[j];
          sacc1[j] += acc1[j] * fv[j];
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      c_al += S;
      ++c_k;
      if (rec_end) {
        c_al = w;
        c_k = 0;
        if (Cq.last) {
          if (ADJ)
            flush_adj(Cq);
          else
            flush(Cq, cpar);
        }
        if (++cr == r_end) {
          done = true;
        } else {
          Cq = recs[cr];
          cpar ^= 1;
          wait_vmcnt<2 * W - 2>();
          lds_barrier();
          read_b();
          // the buffer of the record just finished is free: copy the record
          // after the new one into it, a whole record ahead of its use
          if (cr + 1 < r_end) {
            __builtin_amdgcn_sched_barrier(0);
            stage(recs[cr + 1], cpar ^ 1);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    }
  };

  stage(Rq, 0);
  if (r_begin + 1 < r_end) stage(recs[r_begin + 1], 1);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < W; ++i) refill(a0[i], a1[i]);
  wait_vmcnt<2 * W>();
  lds_barrier();
  read_b();
  // The loop leaves only at the end of the unrolled body (steps after the
  // last one consume nothing and refill from the zero page): an exit from
  // inside the body would be routed through the loop latch by the control
  // flow structurizer, and the compiler's waits at the loop head would then
  // assume that the ring holds the loads of a single step.
  do {
#pragma unroll
    for (int i = 0; i < W; ++i) {
      consume(a0[i], a1[i]);
      refill(a0[i], a1[i]);
    }
  } while (!done);
  wait_vmcnt<0>();
}

// ---------------------------------------------------------------------------
// DIS forward: each wave owns one 16-datapoint block of the item.
// ---------------------------------------------------------------------------
template <int DT, int NT>
__global__ void __launch_bounds__(kThreads)
    dis_fwd_kernel(const FwdItem *__restrict__ items, const SegRef *__restrict__ segs,
                   const GroupDesc *__restrict__ gd, const u32x4 *__restrict__ bop,
                   float *__restrict__ part, const u32x4 *zp) {
  constexpr int RP = 16 * NT;
  extern __shared__ u32x4 lds[];
  const FwdItem it = items[blockIdx.x];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const bool active = w < it.nblk;
  const int bl = it.block0 + w;
  const int nv = active ? min(16, it.ndata - 16 * bl) : 0;
  f32x4 sacc[NT];
  zero(sacc);
  // the tile of the next group is loaded while the current one is multiplied
  u32x4 a0[kTMax], a1[kTMax];
  auto fetch = [&](u32x4 (&a)[kTMax], int s) {
    const SegRef sr = segs[s < it.seg1 ? s : it.seg0];
    const bool in = active && s < it.seg1;
    load_a(a, in ? (const u32x4 *)sr.base + (size_t)bl * sr.KE * 16 : zp, in ? nv : 0, sr.KE, zp);
  };
  auto step = [&](const u32x4 (&a)[kTMax], int s) {
    const SegRef sr = segs[s];
    const int T = (sr.KE + 3) >> 2;
    __syncthreads();
    copy_b(lds, bop + gd[sr.gdesc].bop_off, 4 * T * RP);
    __syncthreads();
    if (active) {
      f32x4 acc[NT];
      zero(acc);
      mma_tile<DT, NT>(a, T, lds, acc);
#pragma unroll
      for (int j = 0; j < NT; ++j) sacc[j] += acc[j];
    }
  };
  fetch(a0, it.seg0);
  fetch(a1, it.seg0 + 1);
  for (int s = it.seg0; s < it.seg1; s += 2) {
    step(a0, s);
    fetch(a0, s + 2);
    if (s + 1 < it.seg1) step(a1, s + 1);
    fetch(a1, s + 3);
  }
  if (active) {
    float *dst = part + (size_t)(it.slot0 + w) * 16 * kRpMax;
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[(4 * g + q) * kRpMax + 16 * j + c] = sacc[j][q];
  }
}

// ---------------------------------------------------------------------------
// Streaming DIS forward.  A workgroup owns a range of 16-datapoint blocks of
// one table; it copies the B operands of all the table's groups into LDS
// once (group after group, so k-step q of a block reads B at 4q), then each
// wave streams whole block rows -- blocks w, w+S, ... of the range, every
// group of a block in turn -- through a ring of W k-steps in registers and
// writes s_i times the dot product straight to the output.  No barrier and
// no partial sums: the contraction of a row is one accumulation chain.
// ---------------------------------------------------------------------------
template <int DT, int NT, int W, int S>
__global__ void __launch_bounds__(64 * S)
    dis_stream_kernel(const DisStreamWG *__restrict__ wgs, const DisGroupRef *__restrict__ groups,
                      const u32x4 *__restrict__ bop, const float *__restrict__ scale_all, int R,
                      int c0, int ncols, float *__restrict__ out, const u32x4 *zp) {
  constexpr int RP = 16 * NT;
  extern __shared__ u32x4 lds[];
  const DisStreamWG wg = wgs[blockIdx.x];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  (void)lane;
  // B of every group, then the scales of the range's datapoints; each
  // thread issues up to eight loads before it stores any
  constexpr int NTHR = 64 * S;
  float *sl = (float *)(lds + 4 * wg.ttot * RP);
  {
    int off = 0;
    for (int gi = wg.g0; gi < wg.g1; ++gi) {
      const int n = 4 * groups[gi].T * RP;
      const u32x4 *src = bop + groups[gi].bop_off;
      for (int i0 = threadIdx.x; i0 < n; i0 += 8 * NTHR) {
        u32x4 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (i0 + k * NTHR < n) v[k] = src[i0 + k * NTHR];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (i0 + k * NTHR < n) lds[off + i0 + k * NTHR] = v[k];
      }
      off += n;
    }
    const int nrow = min(16 * wg.nblk, wg.ndata - 16 * wg.block0);
    const float *ssrc = scale_all + wg.orow0 + 16 * wg.block0;
    for (int i0 = threadIdx.x; i0 < nrow; i0 += 8 * NTHR) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (i0 + k * NTHR < nrow) v[k] = ssrc[i0 + k * NTHR];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (i0 + k * NTHR < nrow) sl[i0 + k * NTHR] = v[k];
    }
  }
  __syncthreads();
  if (w >= wg.nblk) return;  // no block for this wave (after the barrier)

  u32x4 a[W];
  f32x4 acc[NT];
  zero(acc);

  // refill cursor: block rb (relative), group rg, k-step rt of the group.
  // The group's tile of the block is read through a buffer descriptor sized
  // to the tile (zeros past the row's end); absent rows (the last block of
  // a table) get an offset beyond the tile, and past the end of the list
  // the descriptor is empty (see had_stream_kernel).
  int rb = w, rg = wg.g0, rt = 0;
  bool r_done = false;
  DisGroupRef G = groups[rg];
  int rnv = min(16, wg.ndata - 16 * (wg.block0 + rb));
  constexpr unsigned kNoRow = 0x80000000u;
  __amdgpu_buffer_rsrc_t rs;
  unsigned vo = 0, ko = 0;
  auto set_tile = [&]() {
    const u32x4 *p = (const u32x4 *)G.base + (size_t)(wg.block0 + rb) * 16 * G.KE;
    rs = __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, r_done ? 0 : G.KE * rnv * 16,
                                           kBufferRsrcWord3);
    ko = 0;
  };
  auto set_lane = [&]() { vo = c < rnv ? (unsigned)(g * rnv + c) * 16u : kNoRow; };
  set_tile();
  set_lane();
  auto refill = [&](u32x4 &x) {
    x = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo + ko, 0, kLoadNT));
    if (!r_done) {
      ko += 64u * rnv;
      if (++rt == G.T) {
        rt = 0;
        if (++rg == wg.g1) {
          rg = wg.g0;
          rb += S;
          if (rb >= wg.nblk) {
            r_done = true;
          } else {
            rnv = min(16, wg.ndata - 16 * (wg.block0 + rb));
            set_lane();
          }
        }
        G = groups[rg];
        set_tile();
      }
    }
  };
  // consume cursor: block cb, k-step q over all groups of the block.  The
  // B fragments of the next k-step are read right after the MFMAs of this
  // one, so their LDS latency overlaps the refill.
  int cb = w, q = 0;
  bool done = false;
  u32x4 b[NT];
  auto read_b = [&]() {
    const u32x4 *bp = lds + (4 * q + g) * RP + c;
#pragma unroll
    for (int j = 0; j < NT; ++j) b[j] = bp[16 * j];
  };
  read_b();
  auto consume = [&](const u32x4 &x) {
    if (done) return;
    // the first k-step of a block starts the accumulators from zero
    if (q == 0) {
#pragma unroll
      for (int j = 0; j < NT; ++j) Mma<DT>::first(x, b[j], acc[j]);
    } else {
#pragma unroll
      for (int j = 0; j < NT; ++j) Mma<DT>::run(x, b[j], acc[j]);
    }
    const bool blk_end = ++q == wg.ttot;
    if (blk_end) q = 0;
    if (!blk_end || cb + S < wg.nblk) read_b();
    __builtin_amdgcn_sched_barrier(0);
    if (blk_end) {
      // the block's outputs through a descriptor over its rows: a fixed
      // number of stores (no branches, so the waits on the ring stay
      // exact); absent rows and columns past the pass get an offset beyond
      // it and the hardware drops them
      const int row0 = 16 * cb;  // first row of the block within the range
      const int nv = min(16, wg.ndata - 16 * (wg.block0 + cb));
      float *ob = out + (size_t)(wg.orow0 + 16 * (wg.block0 + cb)) * R + c0;
      const __amdgpu_buffer_rsrc_t rso =
          __builtin_amdgcn_make_buffer_rsrc((void *)ob, (short)0, 16 * R * 4, kBufferRsrcWord3);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 4 * g + e;
        const float sc = sl[row0 + min(r, nv - 1)];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const bool ok = r < nv && 16 * j + c < ncols;
          const unsigned off = ok ? (unsigned)(r * R + 16 * j + c) * 4u : kNoRow;
          // the builtin takes the 32 bits as an unsigned integer
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, sc * acc[j][e]), rso, off, 0, 0);
        }
      }
      cb += S;
      if (cb >= wg.nblk) done = true;
    }
  };
#pragma unroll
  for (int i = 0; i < W; ++i) refill(a[i]);
  // single exit at the end of the unrolled body (see had_stream_kernel)
  do {
#pragma unroll
    for (int i = 0; i < W; ++i) {
      consume(a[i]);
      refill(a[i]);
    }
  } while (!done);
  wait_vmcnt<0>();
}

// ---------------------------------------------------------------------------
// Hadronic adjoint: H = Shat f per (block, alpha) tile, weighted by
// W[i,r] = gbar[i,r] s_i and summed over the tile's datapoints.
// ---------------------------------------------------------------------------
template <int DT, int NT>
__device__ __forceinline__ void had_adj_tile(const u32x4 (&a)[kTMax], int T,
                                             const u32x4 *__restrict__ lb,
                                             const float *__restrict__ wl, float *__restrict__ grow) {
  constexpr int RP = 16 * NT;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  f32x4 acc[NT];
  zero(acc);
  mma_tile<DT, NT>(a, T, lb, acc);
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int col = 16 * j + c;
    float v = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) v += acc[j][q] * wl[(4 * g + q) * RP + col];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (g == 0) grow[col] += v;
  }
}

template <int DT, int NT, int S>
__global__ void __launch_bounds__(64 * S)
    had_adj_kernel(const HadAdjItem *__restrict__ items, const SegRef *__restrict__ segs,
                   const GroupDesc *__restrict__ gd, const u32x4 *__restrict__ bop,
                   const float *__restrict__ gout, const float *__restrict__ scale_all, int R,
                   int c0, int ncols, int nx, float *__restrict__ apart, const u32x4 *zp) {
  constexpr int RP = 16 * NT;
  extern __shared__ u32x4 lds[];
  const HadAdjItem it = items[blockIdx.x];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const SegRef sr = segs[it.seg];
  const int KE = sr.KE, T = (KE + 3) >> 2;
  u32x4 *lb = lds;
  float *gacc = (float *)(lds + 4 * T * RP);  // [nx][RP]
  float *wl = gacc + nx * RP;                  // [16][RP]
  constexpr int NTHR = 64 * S;
  {
    const u32x4 *src = bop + gd[sr.gdesc].bop_off;
    for (int i = threadIdx.x; i < 4 * T * RP; i += NTHR) lb[i] = src[i];
  }
  for (int i = threadIdx.x; i < nx * RP; i += NTHR) gacc[i] = 0.f;
  u32x4 a0[kTMax], a1[kTMax];
  for (int bl = it.block0; bl < it.block1; ++bl) {
    const int nv = min(16, it.ndata - 16 * bl);
    const u32x4 *blk = (const u32x4 *)sr.base + (size_t)bl * nx * KE * 16;
    auto fetch = [&](u32x4 (&a)[kTMax], int al) {
      const bool in = al < nx;
      load_a(a, in ? blk + (size_t)al * KE * nv : zp, in ? nv : 0, KE, zp);
    };
    fetch(a0, w);
    fetch(a1, w + S);
    __syncthreads();
    for (int i = threadIdx.x; i < 16 * RP; i += NTHR) {
      const int row = i / RP, col = i - row * RP;
      float v = 0.f;
      if (row < nv && col < ncols) {
        const size_t gi = (size_t)it.wrow0 + 16 * bl + row;
        v = gout[gi * R + c0 + col] * scale_all[gi];
      }
      wl[i] = v;
    }
    __syncthreads();
    for (int al = w; al < nx; al += 2 * S) {
      had_adj_tile<DT, NT>(a0, T, lb, wl, gacc + al * RP);
      fetch(a0, al + 2 * S);
      if (al + S < nx) had_adj_tile<DT, NT>(a1, T, lb, wl, gacc + (al + S) * RP);
      fetch(a1, al + 3 * S);
    }
  }
  __syncthreads();
  float *dst = apart + (size_t)it.slot * nx * kRpMax;
  for (int i = threadIdx.x; i < nx * RP; i += NTHR) {
    const int row = i / RP, col = i - row * RP;
    dst[row * kRpMax + col] = gacc[i];
  }
}

// ---------------------------------------------------------------------------
// DIS adjoint on the transposed table: one 16-row tile of (flavour, x) rows
// per wave, contraction over a chunk of datapoints with B = W.
// ---------------------------------------------------------------------------
template <int DT, int NT>
__global__ void __launch_bounds__(kThreads)
    dis_adj_kernel(const DisAdjItem *__restrict__ items, const GroupDesc *__restrict__ gd,
                   const u32x4 *__restrict__ bop, float *__restrict__ apart, const u32x4 *zp) {
  constexpr int RP = 16 * NT;
  extern __shared__ u32x4 lds[];
  const DisAdjItem it = items[blockIdx.x];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int KE = it.KE, T = (KE + 3) >> 2;
  const bool active = w < it.ntile;
  const int tile = it.tile0 + w;
  const int nv = active ? min(16, it.nrows - 16 * tile) : 0;
  u32x4 a[kTMax];
  load_a(a, active ? (const u32x4 *)it.base + (size_t)tile * 16 * KE : zp, nv, KE, zp);
  copy_b(lds, bop + gd[it.gdesc].bop_off, 4 * T * RP);
  __syncthreads();
  if (active) {
    f32x4 acc[NT];
    zero(acc);
    mma_tile<DT, NT>(a, T, lds, acc);
    float *dst = apart + (size_t)(it.slot0 + w) * 16 * kRpMax;
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[(4 * g + q) * kRpMax + 16 * j + c] = acc[j][q];
  }
}

// ---------------------------------------------------------------------------
// Reductions in a fixed order
// ---------------------------------------------------------------------------
template <int V>
__global__ void __launch_bounds__(kThreads)
    fwd_reduce_kernel(const RedBlock *__restrict__ blocks, const int32_t *__restrict__ slot_idx,
                      const float *__restrict__ part, const float *__restrict__ scale_all,
                      float factor, int R, int c0, int ncols, float *__restrict__ out) {
  // grid: x = chunk of kThreads groups of V adjacent outputs of the block,
  // y = output block.  V = 4 needs ncols, R and c0 multiples of 4 (and an
  // aligned output): then every access is 16 bytes wide.  Each output is
  // the same sum either way: its slots in list order.
  typedef float vec __attribute__((ext_vector_type(V)));
  const RedBlock b = blocks[blockIdx.y];
  const int nc = ncols / V;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= b.nv * nc) return;
  const int row = i / nc, col = (i - row * nc) * V;
  const float *p = part + row * kRpMax + col;
  auto at = [&](int slot) { return *(const vec *)(p + (size_t)slot * 16 * kRpMax); };
  const int orow = b.orow + row;
  const float sc = factor * scale_all[orow];
  const int n = b.k1 - b.k0;
  vec acc = vec(0.f);
  if (n > 0) {
    // the first slots are held in the block record itself; their loads are
    // issued together, unconditionally (past the block's count they re-read
    // its first slot and are not added)
    const int ni = n < kRedInline ? n : kRedInline;
    vec v[kRedInline];
#pragma unroll
    for (int q = 0; q < kRedInline; ++q) v[q] = at(q < ni ? b.slot[q] : b.slot[0]);
#pragma unroll
    for (int q = 0; q < kRedInline; ++q) acc = q < ni ? acc + v[q] : acc;
    for (int k = b.k0 + ni; k < b.k1; ++k) acc += at(slot_idx[k]);
  }
  *(vec *)(out + (size_t)orow * R + c0 + col) = sc * acc;
}

// One output row (flavour, x) per workgroup: kAdjRedRuns groups of 128
// threads (one per column) each add a contiguous run of the row's slots in
// list order, issuing the loads eight at a time; the runs' sums are then
// added in run order.  A fixed order either way.
constexpr int kAdjRedRuns = 4;
__global__ void __launch_bounds__(128 * kAdjRedRuns)
    adj_reduce_kernel(const int32_t *__restrict__ row_ptr, const int64_t *__restrict__ entry,
                      const float *__restrict__ apart, int R, int c0, int ncols, int accumulate,
                      float *__restrict__ g) {
  static_assert(kRpMax <= 128, "one thread per column");
  __shared__ float run_sum[kAdjRedRuns][128];
  const int o = blockIdx.x;
  const int k0 = row_ptr[o], k1 = row_ptr[o + 1];
  const int col = threadIdx.x & 127;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 7);
  const int n = k1 - k0, per = (n + kAdjRedRuns - 1) / kAdjRedRuns;
  const int ka = k0 + min(n, q * per), kb = k0 + min(n, (q + 1) * per);
  float acc = 0.f;
  if (col < ncols) {
    int k = ka;
    for (; k + 8 <= kb; k += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = apart[entry[k + u] + col];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; k < kb; ++k) acc += apart[entry[k] + col];
  }
  run_sum[q][col] = acc;
  __syncthreads();
  if (q == 0 && col < ncols) {
    float sum = run_sum[0][col];
#pragma unroll
    for (int r = 1; r < kAdjRedRuns; ++r) sum += run_sum[r][col];
    float *p = g + (size_t)o * R + c0 + col;
    *p = accumulate ? *p + sum : sum;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {

#define FK_DISPATCH_NT(call)            \
  switch (L.nt) {                       \
    case 1: call(1); break;             \
    case 2: call(2); break;             \
    case 4: call(4); break;             \
    case 7: call(7); break;             \
    case 8: call(8); break;             \
    default: return hipErrorInvalidValue; \
  }

#define FK_DISPATCH_DT(call_dt)                          \
  switch (L.dtype) {                                     \
    case FK_F32: call_dt(FK_F32); break;                 \
    case FK_BF16: call_dt(FK_BF16); break;               \
    case FK_FP8E4M3: call_dt(FK_FP8E4M3); break;         \
    default: return hipErrorInvalidValue;                \
  }

template <typename KernT>
hipError_t set_lds(KernT kern, size_t bytes) {
  if (bytes > 65536)
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
  return hipSuccess;
}

}  // namespace

hipError_t launch_stage_b(const ConvLaunch &L, const GroupDesc *d_gd, const int32_t *rowtab,
                          int ngd, const float *pdf,
                          const float *gout, const float *scale_all, uint4 *bop, int *counter,
                          float *fstage, int nflav, int nx, const int32_t *wrow, float *wstage,
                          int nwpair) {
  if (ngd <= 0) return hipSuccess;
  if (fstage && wstage) return hipErrorInvalidValue;
  const int RP = 16 * L.nt;
  // one thread per staged unit (a group's B has at most 4*kTMax*RP units)
  int units = 4 * kTMax * RP;
  if (fstage) units = std::max(units, nx * RP);
  const int gx = (units + kThreads - 1) / kThreads;
  int rows = ngd + (fstage ? nflav : 0);
  if (wstage)
    rows += (int)(((size_t)nwpair * RP * kAdjWRow + (size_t)gx * kThreads - 1) /
                  ((size_t)gx * kThreads));
  const dim3 grid(gx, rows);
#define FK_STAGE(DT)                                                                          \
  hipLaunchKernelGGL(stage_b_kernel<DT>, grid, dim3(kThreads), 0, L.stream, d_gd, rowtab, ngd, \
                     pdf, gout, scale_all, L.R, L.c0, L.ncols, RP, (u32x4 *)bop, counter,      \
                     fstage, nx, wrow, wstage, nwpair)
  FK_DISPATCH_DT(FK_STAGE);
#undef FK_STAGE
  return hipGetLastError();
}

hipError_t launch_had_fwd(const ConvLaunch &L, const FwdItem *items, int nitems, const SegRef *segs,
                          const GroupDesc *gd, const uint4 *bop, const float *pdf, int nx,
                          int lds_units, float *part, int *counter, int grid) {
  if (nitems <= 0) return hipSuccess;
  // B operand, or the combine buffer [2 blocks][4 waves][16][RP] floats
  const size_t lds = std::max((size_t)lds_units * 16, (size_t)2 * kWaves * 16 * 16 * L.nt * 4);
  grid = std::max(1, std::min(grid, nitems));
  hipError_t err = hipSuccess;
#define FK_HF(NT)                                                                            \
  {                                                                                          \
    auto k = had_fwd_kernel<DTV, NT>;                                                        \
    if ((err = set_lds(k, lds)) != hipSuccess) return err;                                   \
    hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, L.stream, items, nitems, segs, gd, \
                       (const u32x4 *)bop, pdf, L.R, L.c0, L.ncols, nx, part,                \
                       (const u32x4 *)L.zero_page, counter);                                 \
  }
#define FK_HF_DT(DT)           \
  {                            \
    constexpr int DTV = DT;    \
    FK_DISPATCH_NT(FK_HF);     \
  }
  FK_DISPATCH_DT(FK_HF_DT);
#undef FK_HF
#undef FK_HF_DT
  return hipGetLastError();
}

size_t had_stream_lds_bytes(int nt, int nx, int maxT, int mode) {
  const int RP = 16 * nt;
  // forward: B operand + PDF rows, or the combine buffer [2][4][16][RP]
  // floats; adjoint: B operand + the weights [RP][kAdjWRow] floats
  int units = mode == kStreamAdj ? 4 * maxT * RP + RP * kAdjWRow / 4
                                 : std::max(4 * maxT * RP + nx * RP / 4, 2 * 4 * 16 * RP / 4);
  units = (units + 63) / 64 * 64;
  const size_t bytes = (size_t)2 * units * 16;
  return bytes <= 163840 ? bytes : 0;
}

hipError_t launch_had_stream(const ConvLaunch &L, const StreamSeg *recs, const int32_t *wg_ptr,
                             int grid, const uint4 *bop, const float *fstage, int nx, int maxT,
                             float *part, int mode) {
  if (grid <= 0) return hipSuccess;
  const size_t lds = had_stream_lds_bytes(L.nt, nx, maxT, mode);
  if (!lds) return hipErrorInvalidValue;
  if (mode == kStreamAdj && nx > 8 * kStreamWaves) return hipErrorInvalidValue;
  const int bufsz = (int)(lds / 32);  // units per buffer
  hipError_t err = hipSuccess;
#define FK_HS_MODE(NT, MODE)                                                                   \
  {                                                                                            \
    auto k = had_stream_kernel<DTV, NT, kStreamW, kStreamWaves, MODE>;                         \
    if ((err = set_lds(k, lds)) != hipSuccess) return err;                                     \
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * kStreamWaves), lds, L.stream, recs, wg_ptr,    \
                       (const u32x4 *)bop, fstage, nx, bufsz, part, (const u32x4 *)L.zero_page); \
  }
#define FK_HS(NT)                         \
  {                                       \
    if (mode == kStreamAdj)               \
      FK_HS_MODE(NT, kStreamAdj)          \
    else                                  \
      FK_HS_MODE(NT, kStreamFwd)          \
  }
#define FK_HS_DT(DT)           \
  {                            \
    constexpr int DTV = DT;    \
    FK_DISPATCH_NT(FK_HS);     \
  }
  FK_DISPATCH_DT(FK_HS_DT);
#undef FK_HS
#undef FK_HS_MODE
#undef FK_HS_DT
  return hipGetLastError();
}

size_t dis_stream_lds_bytes(int nt, int ttot_max) {
  const size_t bytes = (size_t)4 * ttot_max * 16 * nt * 16 + (size_t)16 * kDisStreamMaxBlk * 4;
  return bytes <= 163840 ? bytes : 0;
}

hipError_t launch_dis_stream(const ConvLaunch &L, const DisStreamWG *wgs, int nwg,
                             const DisGroupRef *groups, const uint4 *bop, const float *scale_all,
                             int ttot_max, float *out) {
  if (nwg <= 0) return hipSuccess;
  const size_t lds = dis_stream_lds_bytes(L.nt, ttot_max);
  if (!lds) return hipErrorInvalidValue;
  hipError_t err = hipSuccess;
#define FK_DS(NT)                                                                              \
  {                                                                                            \
    auto k = dis_stream_kernel<DTV, NT, kDisStreamW, kDisStreamWaves>;                         \
    if ((err = set_lds(k, lds)) != hipSuccess) return err;                                     \
    hipLaunchKernelGGL(k, dim3(nwg), dim3(64 * kDisStreamWaves), lds, L.stream, wgs, groups,   \
                       (const u32x4 *)bop, scale_all, L.R, L.c0, L.ncols, out,                 \
                       (const u32x4 *)L.zero_page);                                            \
  }
#define FK_DS_DT(DT)           \
  {                            \
    constexpr int DTV = DT;    \
    FK_DISPATCH_NT(FK_DS);     \
  }
  FK_DISPATCH_DT(FK_DS_DT);
#undef FK_DS
#undef FK_DS_DT
  return hipGetLastError();
}

hipError_t launch_dis_fwd(const ConvLaunch &L, const FwdItem *items, int nitems, const SegRef *segs,
                          const GroupDesc *gd, const uint4 *bop, int lds_units, float *part) {
  if (nitems <= 0) return hipSuccess;
  const size_t lds = (size_t)lds_units * 16;
  hipError_t err = hipSuccess;
#define FK_DF(NT)                                                                          \
  {                                                                                        \
    auto k = dis_fwd_kernel<DTV, NT>;                                                      \
    if ((err = set_lds(k, lds)) != hipSuccess) return err;                                 \
    hipLaunchKernelGGL(k, dim3(nitems), dim3(kThreads), lds, L.stream, items, segs, gd,    \
                       (const u32x4 *)bop, part, (const u32x4 *)L.zero_page);              \
  }
#define FK_DF_DT(DT)           \
  {                            \
    constexpr int DTV = DT;    \
    FK_DISPATCH_NT(FK_DF);     \
  }
  FK_DISPATCH_DT(FK_DF_DT);
#undef FK_DF
#undef FK_DF_DT
  return hipGetLastError();
}

hipError_t launch_fwd_reduce(const ConvLaunch &L, const RedBlock *blocks, int nblocks,
                             const int32_t *slot_idx, const float *part, const float *scale_all,
                             float factor, float *out) {
  if (nblocks <= 0) return hipSuccess;
  const bool v4 = L.ncols % 4 == 0 && L.R % 4 == 0 && L.c0 % 4 == 0 && (uintptr_t)out % 16 == 0;
  if (v4)
    hipLaunchKernelGGL(fwd_reduce_kernel<4>,
                       dim3((16 * L.ncols / 4 + kThreads - 1) / kThreads, nblocks), dim3(kThreads),
                       0, L.stream, blocks, slot_idx, part, scale_all, factor, L.R, L.c0, L.ncols,
                       out);
  else
    hipLaunchKernelGGL(fwd_reduce_kernel<1>, dim3((16 * L.ncols + kThreads - 1) / kThreads, nblocks),
                       dim3(kThreads), 0, L.stream, blocks, slot_idx, part, scale_all, factor, L.R,
                       L.c0, L.ncols, out);
  return hipGetLastError();
}

hipError_t launch_had_adj(const ConvLaunch &L, const HadAdjItem *items, int nitems,
                          const SegRef *segs, const GroupDesc *gd, const uint4 *bop,
                          const float *gout, const float *scale_all, int nx, int lds_units,
                          float *apart) {
  if (nitems <= 0) return hipSuccess;
  const int RP = 16 * L.nt;
  const size_t lds = (size_t)lds_units * 16 + (size_t)(nx + 16) * RP * 4;
  hipError_t err = hipSuccess;
#define FK_HA(NT)                                                                              \
  {                                                                                            \
    auto k = had_adj_kernel<DTV, NT, kAdjWaves>;                                               \
    if ((err = set_lds(k, lds)) != hipSuccess) return err;                                     \
    hipLaunchKernelGGL(k, dim3(nitems), dim3(64 * kAdjWaves), lds, L.stream, items, segs, gd,  \
                       (const u32x4 *)bop, gout, scale_all, L.R, L.c0, L.ncols, nx, apart,     \
                       (const u32x4 *)L.zero_page);                                            \
  }
#define FK_HA_DT(DT)           \
  {                            \
    constexpr int DTV = DT;    \
    FK_DISPATCH_NT(FK_HA);     \
  }
  FK_DISPATCH_DT(FK_HA_DT);
#undef FK_HA
#undef FK_HA_DT
  return hipGetLastError();
}

hipError_t launch_dis_adj(const ConvLaunch &L, const DisAdjItem *items, int nitems,
                          const GroupDesc *gd, const uint4 *bop, int lds_units, float *apart) {
  if (nitems <= 0) return hipSuccess;
  const size_t lds = (size_t)lds_units * 16;
  hipError_t err = hipSuccess;
#define FK_DA(NT)                                                                          \
  {                                                                                        \
    auto k = dis_adj_kernel<DTV, NT>;                                                      \
    if ((err = set_lds(k, lds)) != hipSuccess) return err;                                 \
    hipLaunchKernelGGL(k, dim3(nitems), dim3(kThreads), lds, L.stream, items, gd,          \
                       (const u32x4 *)bop, apart, (const u32x4 *)L.zero_page);             \
  }
#define FK_DA_DT(DT)           \
  {                            \
    constexpr int DTV = DT;    \
    FK_DISPATCH_NT(FK_DA);     \
  }
  FK_DISPATCH_DT(FK_DA_DT);
#undef FK_DA
#undef FK_DA_DT
  return hipGetLastError();
}

hipError_t launch_adj_reduce(const ConvLaunch &L, int nrows_out, const int32_t *row_ptr,
                             const int64_t *entry_off, const float *apart, int accumulate,
                             float *g) {
  if (nrows_out <= 0) return hipSuccess;
  if (L.ncols > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(adj_reduce_kernel, dim3(nrows_out), dim3(128 * kAdjRedRuns), 0, L.stream,
                     row_ptr, entry_off, apart, L.R, L.c0, L.ncols, accumulate, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Error of a reduced-precision result against a reference, per replica
// column: out[2 r] = sum_i (y[i,r] - ref[i,r])^2, out[2 r + 1] = sum_i
// ref[i,r]^2, in FP64.  One wave per column, lanes stride the rows, a fixed
// tree across the wave.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64)
    col_err_kernel(const float *__restrict__ y, const float *__restrict__ ref, int N, int R,
                   double *__restrict__ out) {
  const int r = blockIdx.x, lane = threadIdx.x;
  double d2 = 0.0, r2 = 0.0;
  for (int i = lane; i < N; i += 64) {
    const double a = ref[(size_t)i * R + r], b = y[(size_t)i * R + r];
    d2 += (b - a) * (b - a);
    r2 += a * a;
  }
  for (int o = 32; o > 0; o >>= 1) {
    d2 += __shfl_xor(d2, o);
    r2 += __shfl_xor(r2, o);
  }
  if (lane == 0) {
    out[2 * r] = d2;
    out[2 * r + 1] = r2;
  }
}

hipError_t launch_col_err(const float *y, const float *ref, int N, int R, double *out,
                          hipStream_t s) {
  if (N <= 0 || R <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(col_err_kernel, dim3(R), dim3(64), 0, s, y, ref, N, R, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free entry point (fk_conv_dis_static): a
// file-scope device array, one copy per GPU, resolved to its device address
// once per device by static_scratch_resolve.  Host code uses only the
// resolved address: the array's name is a host-side stand-in.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_resolve(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_dev[device] = p;
  return hipSuccess;
}

void *static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_dev[device];
}

}  // namespace fk
