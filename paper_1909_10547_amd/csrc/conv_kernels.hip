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
// All partial sums are written to slots and reduced in a fixed order, so
// results are bitwise reproducible and independent of batch composition.
#include <algorithm>

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
};

// Table pointers come from descriptors in memory, so the compiler cannot
// infer their address space and would emit flat loads, which count against
// the LDS wait counter as well: every LDS read of the B operand would then
// wait for the in-flight HBM prefetch.  The tables live in global memory.
typedef const __attribute__((address_space(1))) u32x4 *gu32x4_ptr;
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
    stage_b_kernel(const GroupDesc *__restrict__ gd, const float *__restrict__ pdf,
                   const float *__restrict__ gout, const float *__restrict__ scale_all, int R,
                   int c0, int ncols, int RP, u32x4 *__restrict__ bop, int *counter) {
  constexpr int E = Mma<DT>::E;
  // the forward kernel that follows on the stream takes items from *counter
  if (counter && blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
  __shared__ int s_row[kMaxSeg], s_start[kMaxSeg + 1];
  const GroupDesc *G = gd + blockIdx.x;
  const int nseg = G->nseg, K = G->K, src_kind = G->src;
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int s = 0; s < nseg; ++s) {
      s_row[s] = G->seg_row[s];
      s_start[s] = acc;
      acc += G->seg_len[s];
    }
    s_start[nseg] = acc;
  }
  __syncthreads();
  const float *src = src_kind == 0 ? pdf : gout;
  const int KEpad = ((G->KE + 3) >> 2) << 2;
  const int units = KEpad * RP;
  u32x4 *dst = bop + G->bop_off;
  for (int idx = threadIdx.x; idx < units; idx += kThreads) {
    const int u = idx / RP, n = idx - u * RP;
    float v[E];
    int s = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = u * E + e;
      float x = 0.f;
      if (k < K && n < ncols) {
        while (s_start[s + 1] <= k) ++s;
        const int row = s_row[s] + (k - s_start[s]);
        x = src[(size_t)row * R + c0 + n];
        if (src_kind == 1) x *= scale_all[row];
      }
      v[e] = x;
    }
    dst[idx] = pack_unit<DT>(v);
  }
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
        p.p0 = base + ((size_t)bl0 * nx * 16 + (size_t)al * nv0) * sr.KE;
        p.p1 = nv1 ? base + ((size_t)(bl0 + 1) * nx * 16 + (size_t)al * nv1) * sr.KE : zp;
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

template <int DT, int NT>
__global__ void __launch_bounds__(kThreads)
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
  copy_b(lb, bop + gd[sr.gdesc].bop_off, 4 * T * RP);
  for (int i = threadIdx.x; i < nx * RP; i += kThreads) gacc[i] = 0.f;
  u32x4 a0[kTMax], a1[kTMax];
  constexpr int S = kWaves;
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
    for (int i = threadIdx.x; i < 16 * RP; i += kThreads) {
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
  for (int i = threadIdx.x; i < nx * RP; i += kThreads) {
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
__global__ void __launch_bounds__(kThreads)
    fwd_reduce_kernel(const RedBlock *__restrict__ blocks, const int32_t *__restrict__ slot_idx,
                      const float *__restrict__ part, const float *__restrict__ scale_all,
                      float factor, int R, int c0, int ncols, float *__restrict__ out) {
  const RedBlock b = blocks[blockIdx.x];
  for (int i = threadIdx.x; i < b.nv * ncols; i += kThreads) {
    const int row = i / ncols, col = i - row * ncols;
    float acc = 0.f;
    for (int k = b.k0; k < b.k1; ++k) acc += part[(size_t)slot_idx[k] * 16 * kRpMax + row * kRpMax + col];
    const int orow = b.orow + row;
    out[(size_t)orow * R + c0 + col] = factor * scale_all[orow] * acc;
  }
}

__global__ void __launch_bounds__(kThreads)
    adj_reduce_kernel(const int32_t *__restrict__ row_ptr, const int64_t *__restrict__ entry,
                      const float *__restrict__ apart, int R, int c0, int ncols, int accumulate,
                      float *__restrict__ g) {
  const int o = blockIdx.x;
  const int k0 = row_ptr[o], k1 = row_ptr[o + 1];
  for (int col = threadIdx.x; col < ncols; col += kThreads) {
    float acc = 0.f;
    for (int k = k0; k < k1; ++k) acc += apart[entry[k] + col];
    float *p = g + (size_t)o * R + c0 + col;
    *p = accumulate ? *p + acc : acc;
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

hipError_t launch_stage_b(const ConvLaunch &L, const GroupDesc *d_gd, int ngd, const float *pdf,
                          const float *gout, const float *scale_all, uint4 *bop, int *counter) {
  if (ngd <= 0) return hipSuccess;
  const int RP = 16 * L.nt;
#define FK_STAGE(DT)                                                                        \
  hipLaunchKernelGGL(stage_b_kernel<DT>, dim3(ngd), dim3(kThreads), 0, L.stream, d_gd, pdf, \
                     gout, scale_all, L.R, L.c0, L.ncols, RP, (u32x4 *)bop, counter)
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
  hipLaunchKernelGGL(fwd_reduce_kernel, dim3(nblocks), dim3(kThreads), 0, L.stream, blocks,
                     slot_idx, part, scale_all, factor, L.R, L.c0, L.ncols, out);
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
    auto k = had_adj_kernel<DTV, NT>;                                                          \
    if ((err = set_lds(k, lds)) != hipSuccess) return err;                                     \
    hipLaunchKernelGGL(k, dim3(nitems), dim3(kThreads), lds, L.stream, items, segs, gd,        \
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
  hipLaunchKernelGGL(adj_reduce_kernel, dim3(nrows_out), dim3(kThreads), 0, L.stream, row_ptr,
                     entry_off, apart, L.R, L.c0, L.ncols, accumulate, g);
  return hipGetLastError();
}

}  // namespace fk
