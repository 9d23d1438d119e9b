// HIP kernels of the lsdm library (gfx950).
//
//  * layout conversion between the caller's block layout and the internal
//    strip layout (gather/scatter of 4x4 sub-blocks);
//  * strip-layout transpose (B^T for products with a transposed B);
//  * the symbolic step generation of product plans;
//  * the truncated block product C = alpha P_C(op(A) B) + beta C on MFMA:
//    one workgroup per group tile of 16 output rows x GJ output column quads,
//    operands staged in LDS, one 16x16 MFMA per active (row quad, column quad)
//    slot and step (FP64, FP32) or per 4 steps (BF16);
//  * the residual-mode FP64 corrections, K assembly (eq. 3) and a
//    bitwise-reproducible compensated FP64 dot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "kernels.h"
#include "plan_common.h"

namespace lsdm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ i64 uniform64(i64 v) {
  int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((i64)hi << 32) | (unsigned)lo;
}

// ---------------------------------------------------------------------------
// fills and conversions
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(T* __restrict__ p, i64 n, T v) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

__device__ __forceinline__ void load4(const float* p, float (&v)[4]) {
  const float4 x = *reinterpret_cast<const float4*>(p);
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
  const double2 x = reinterpret_cast<const double2*>(p)[0], y = reinterpret_cast<const double2*>(p)[1];
  v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
}

__device__ __forceinline__ void store4(float* p, const float (&v)[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store4(unsigned short* p, const unsigned short (&v)[4]) {
  *reinterpret_cast<ushort4*>(p) = make_ushort4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store4(double* p, const double (&v)[4]) {
  reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
}

// one thread per row of every 4x4 sub-block of the map; the row is written
// whole (its padding columns as zero, which they hold anyway)
template <class T>
__global__ void k_user_to_strip(const double* __restrict__ user, T* __restrict__ strip, const i64* __restrict__ su,
                                const i64* __restrict__ ss, const i32* __restrict__ sh, i64 nsub, double scale) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nsub * 4; g += (i64)gridDim.x * blockDim.x) {
    const i64 sb = g >> 2;
    const int r = (int)(g & 3);
    const int shape = sh[sb], rows = shape & 255, cols = (shape >> 8) & 255, stride = shape >> 16;
    if (r >= rows) continue;
    const double* u = user + su[sb] + (i64)r * stride;
    T v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = c < cols ? (T)(scale * u[c]) : (T)0;
    store4(strip + ss[sb] + r * 4, v);
  }
}

// one thread per row of every 4x4 sub-block of the map
template <class T>
__global__ void k_strip_to_user(const T* __restrict__ strip, double* __restrict__ user, const i64* __restrict__ su,
                                const i64* __restrict__ ss, const i32* __restrict__ sh, i64 nsub) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nsub * 4; g += (i64)gridDim.x * blockDim.x) {
    const i64 sb = g >> 2;
    const int r = (int)(g & 3);
    const int shape = sh[sb], rows = shape & 255, cols = (shape >> 8) & 255, stride = shape >> 16;
    if (r >= rows) continue;
    T v[4];
    load4(strip + ss[sb] + r * 4, v);
    double* u = user + su[sb] + (i64)r * stride;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < cols) u[c] = (double)v[c];
  }
}

// out = in^T in strip layout: block t of strip s is the transpose of the block
// at value offset mirror[4s+t] of `in` (zero when the mirror is absent)
template <class T>
__global__ void k_transpose_strips(const T* __restrict__ in, T* __restrict__ out, const i64* __restrict__ mirror,
                                   i64 nstrips) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nstrips * 64; g += (i64)gridDim.x * blockDim.x) {
    const i64 s = g >> 6;
    const int t = (int)((g >> 4) & 3), r = (int)((g >> 2) & 3), c = (int)(g & 3);
    const i64 m = mirror[4 * s + t];
    out[g] = m < 0 ? (T)0 : in[m + c * 4 + r];
  }
}

// dE/dL of symmetric mode in the caller's layout, one thread per row of every
// 4x4 sub-block: Lbar + V + V^T, where Lbar holds only the kept half (a block
// of the dropped half is the transpose of its mirror, as the mirror fill
// would make it; zero when the mirror is absent) and V is whole.  The sums
// are formed in the order that adding V + V^T to the kept half and then
// mirroring it forms them, so either route gives the same bits.
template <class T>
__global__ void k_sym_grad_to_user(const T* __restrict__ Lb, const T* __restrict__ V, double* __restrict__ user,
                                   const i64* __restrict__ su, const i64* __restrict__ ss,
                                   const i32* __restrict__ sh, i64 nsub, const i64* __restrict__ mirror,
                                   const i32* __restrict__ srow, const i32* __restrict__ squad,
                                   const i32* __restrict__ simg) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nsub * 4; g += (i64)gridDim.x * blockDim.x) {
    const i64 sb = g >> 2;
    const int r = (int)(g & 3);
    const int shape = sh[sb], rows = shape & 255, cols = (shape >> 8) & 255, stride = shape >> 16;
    if (r >= rows) continue;
    const i64 so = ss[sb];                  // strip-layout offset of the block's (0, 0)
    const i64 s = so >> 6;
    const int t = (int)((so >> 4) & 3);
    const i32 p = srow[s], q = squad[s], n = simg[s];
    const bool dropped = !keep_strip(p, q, n) || (q == (p >> 2) && n == IMG0 && 4 * q + t < p);
    const i64 m = mirror[4 * s + t];
    T x[4] = {(T)0, (T)0, (T)0, (T)0};
    if (!dropped) {
      T v[4], l[4];
      load4(V + so + r * 4, v);
      load4(Lb + so + r * 4, l);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T w = v[c];
        if (m >= 0) w += V[m + c * 4 + r];
        x[c] = l[c] + w;
      }
    } else if (m >= 0) {
      // the mirror block (kept) after its own update, transposed: row r here
      // is column r there
      const i64 ms = m >> 6;
      const int mt = (int)((m >> 4) & 3);
      const i64 mm = mirror[4 * ms + mt];   // the mirror's mirror: this block
      T vb[4] = {(T)0, (T)0, (T)0, (T)0};
      if (mm >= 0) load4(V + mm + r * 4, vb);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T w = V[m + c * 4 + r];
        if (mm >= 0) w += vb[c];
        x[c] = Lb[m + c * 4 + r] + w;
      }
    }
    double* u = user + su[sb] + (i64)r * stride;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < cols) u[c] = (double)x[c];
  }
}


// The dropped half of a symmetric result from its kept half, in place: one
// thread per row of a block to fill (the list holds strip << 4 | block mask),
// which gathers the matching column of the mirror block.  The mirror of a
// filled block is never filled itself: blocks outside keep_strip mirror into
// kept strips, and in a row's own quad at image 0 the blocks below the
// diagonal mirror to blocks above it.  Absent blocks of a filled strip are
// written as zero.
template <class T>
__global__ void k_sym_fill(T* data, const i64* __restrict__ fill, const i64* __restrict__ mirror, i64 nfill) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nfill * 16; g += (i64)gridDim.x * blockDim.x) {
    const i64 e = fill[g >> 4];
    const int t = (int)((g >> 2) & 3), r = (int)(g & 3);
    if (!((e >> t) & 1)) continue;
    const i64 s = e >> 4;
    const i64 m = mirror[4 * s + t];
    T v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = m < 0 ? (T)0 : data[m + c * 4 + r];
    store4(data + s * 64 + t * 16 + r * 4, v);   // one 16- or 32-byte store
  }
}

// Mirror-write words of a symmetric pattern (lsdm_pattern::d_mirw), one
// thread per block slot of every strip; dropped strips get 0.
__global__ void k_mirw(const i32* __restrict__ srow, const i32* __restrict__ squad, const i32* __restrict__ simg,
                       const uint8_t* __restrict__ smask, const i64* __restrict__ mirror, i32* __restrict__ mw,
                       i64 nstrips) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nstrips * 4; g += (i64)gridDim.x * blockDim.x) {
    const i64 st = g >> 2;
    const int t = (int)(g & 3);
    const i32 q = srow[st], cq = squad[st], n = simg[st];
    i32 w = 0;
    if (keep_strip(q, cq, n)) {
      const bool own = cq == (q >> 2) && n == IMG0;
      const bool present = (smask[st] >> t) & 1;
      const i32 qcol = 4 * cq + t;
      const bool self = !(own && qcol < q && present);
      const i64 m = mirror[g];
      const bool wm = present && !(own && qcol <= q) && m >= 0;
      w = (i32)(((wm ? (m >> 4) + 1 : 0) << 1) | (self ? 1 : 0));
    }
    mw[g] = w;
  }
}

// ---------------------------------------------------------------------------
// Dense 16x16x4 MFMA forms used by the product kernels: one instruction per
// active column quad covers the 4 rows of a row quad at once.
//   f32 16x16x4: lane l holds A[l%16][l/16] and B[l/16][l%16]; D[4(l/16)+v][l%16]
//   f64 16x16x4: same A and B; D[4v + l/16][l%16]          (measured on gfx950)
// ---------------------------------------------------------------------------
template <class T> struct Mma16;
template <> struct Mma16<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mma16<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// ---------------------------------------------------------------------------
// BF16 operand copies: FP32 strips rounded to bf16 (nearest even), either in
// the strip layout (row-major blocks, "R") or with every 4x4 block transposed
// (column-major blocks, "C").
// ---------------------------------------------------------------------------
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
  return (unsigned short)(u >> 16);
}

// caller's block layout (FP64) -> bf16 strips, rounded through FP32 as the
// FP32 strips would be: R keeps the layout, C transposes every 4x4 block.
// One thread per row of every sub-block; the row's padding columns are
// written as zero, which they hold anyway.
__global__ void k_user_to_bf16(const double* __restrict__ user, unsigned short* __restrict__ outR,
                               unsigned short* __restrict__ outC, const i64* __restrict__ su,
                               const i64* __restrict__ ss, const i32* __restrict__ sh, i64 nsub) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nsub * 4; g += (i64)gridDim.x * blockDim.x) {
    const i64 sb = g >> 2;
    const int r = (int)(g & 3);
    const int shape = sh[sb], rows = shape & 255, cols = (shape >> 8) & 255, stride = shape >> 16;
    if (r >= rows) continue;
    const double* u = user + su[sb] + (i64)r * stride;
    unsigned short v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = c < cols ? bf16_rne((float)u[c]) : (unsigned short)0;
    const i64 o = ss[sb];
    if (outR) store4(outR + o + r * 4, v);
    if (outC)
#pragma unroll
      for (int c = 0; c < 4; ++c) outC[o + c * 4 + r] = v[c];
  }
}

// fp32 strips -> bf16 copies: R keeps the layout, C transposes every 4x4 block
__global__ void k_to_bf16(const float* __restrict__ in, unsigned short* __restrict__ outR,
                          unsigned short* __restrict__ outC, i64 n) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < n; g += (i64)gridDim.x * blockDim.x) {
    const unsigned short v = bf16_rne(in[g]);
    if (outR) outR[g] = v;
    if (outC) {
      const int e = (int)(g & 15), r = e >> 2, c = e & 3;
      outC[(g & ~(i64)15) + c * 4 + r] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// plan steps (symbolic pass, on the GPU): one wavefront per group tile; lane
// (entry el, column jq) evaluates one inner entry against one output column
// quad; the slot bits of an entry are OR-ed over its GJ lanes, active entries
// become steps in inner-list order.  Count pass: steps per tile and the useful
// work (integer atomics, so the totals are exact and order independent).  Fill
// pass: writes the step records from the tile's first step.  A step names
// only the operands it uses: a B strip whose column quad has no active slot,
// and an A block whose row has none, are recorded as absent (-1), so the
// product kernels do not fetch them (they could only meet masked outputs or
// zero blocks).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_plan_gsteps(const GTile* __restrict__ tiles, i64 ntiles,
                                                     const GKEnt* __restrict__ kent, const i64* __restrict__ kbeg,
                                                     PlanView v, int fill, i32* __restrict__ counts,
                                                     GStep* __restrict__ steps,
                                                     unsigned long long* __restrict__ work) {
  constexpr int EPI = 64 / GJ;
  const int lane = threadIdx.x & 63;
  const i64 wave0 = (i64)blockIdx.x * 4 + (threadIdx.x >> 6);
  const i64 nw = (i64)gridDim.x * 4;
  const int jq = lane % GJ, el = lane / GJ;
  for (i64 t = wave0; t < ntiles; t += nw) {
    const GTile& tl = tiles[t];
    const i64 ck = gtile_column_key(v, tl, jq);
    const i64 kb = kbeg[tl.group], ke = kbeg[tl.group + 1];
    i64 pos = tl.step0;
    int cnt = 0;
    uint64_t fl = 0, tr = 0;
    for (i64 e0 = kb; e0 < ke; e0 += EPI) {
      const i64 e = e0 + el;
      i32 b = -1;
      uint32_t m[GQ];
#pragma unroll
      for (int w = 0; w < GQ; ++w) m[w] = 0;
      if (e < ke) gslot_work(v, tl, kent[e], jq, ck, &b, m, &fl, &tr);
      // this lane's column has an active slot: its B strip is used
      if ((m[0] | m[1] | m[2] | m[3]) == 0u) b = -1;
      static_assert(GQ == 4, "column activity test");
      uint32_t any = 0;
#pragma unroll
      for (int w = 0; w < GQ; ++w) {
#pragma unroll
        for (int o = 1; o < GJ; o <<= 1) m[w] |= (uint32_t)__shfl_xor((int)m[w], o);
        any |= m[w];
      }
      const bool active = any != 0u;
      const unsigned long long vote = __ballot(active && jq == 0);
      const unsigned long long bvote = __ballot(b >= 0);
      if (fill && active) {
        const int before = __popcll(vote & ((1ull << (el * GJ)) - 1ull));
        int* sp = reinterpret_cast<int*>(steps + pos + before);
        sp[GROWS + jq] = b;
        if (jq == 0) {
          const GKEnt& ent = kent[e];
          uint32_t rows = 0;
#pragma unroll
          for (int r = 0; r < GROWS; ++r) {
            // the row has an active slot in some column quad: its A block is used
            const bool used = ((m[r >> 2] >> (GJ * (r & 3))) & ((1u << GJ) - 1u)) != 0u;
            const i32 a = used ? ent.a[r] : -1;
            sp[r] = a;
            rows |= (a >= 0 ? 1u : 0u) << r;
          }
#pragma unroll
          for (int w = 0; w < GQ; ++w) sp[GROWS + GJ + w] = (int)m[w];
          sp[GROWS + GJ + GQ] = (int)rows;
          sp[GROWS + GJ + GQ + 1] = (int)((bvote >> (el * GJ)) & ((1ull << GJ) - 1ull));
#pragma unroll
          for (int z = GROWS + GJ + GQ + 2; z < 32; ++z) sp[z] = 0;
        }
      }
      const int nv = __popcll(vote);
      pos += nv;
      cnt += nv;
    }
    if (!fill) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        fl += (uint64_t)__shfl_xor((long long)fl, o);
        tr += (uint64_t)__shfl_xor((long long)tr, o);
      }
      if (lane == 0) {
        counts[t] = cnt;
        atomicAdd(work, (unsigned long long)fl);
        atomicAdd(work + 1, (unsigned long long)tr);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Group-tile product on the dense 16x16x4 MFMA with LDS staging.
//
// A workgroup of GQ = 4 wavefronts owns one group tile at a time: 16 output
// rows (wavefront w: row quad w) x GJ column quads.  The tile's steps are
// processed in batches of SB.  Every batch's step records and operands (per
// step the 16 A blocks of the group's rows and the GJ B strips, each fetched
// once for all four wavefronts) are copied from global memory straight into
// LDS (global_load_lds, 16 bytes per lane, 1 KB per instruction), with no
// register staging.  Software pipeline with lookahead DA, one workgroup
// barrier per batch q:
//   top of batch q (after waiting for this wavefront's copies of operands q
//   and records q+DA, and the barrier): every wavefront is done with batch
//   q-1, so its LDS slots may be refilled;
//   copy records q+DA+1 (wavefront 0) and operands q+DA (addresses from
//   records q+DA in LDS), then run the MFMAs of batch q from LDS.
// The copies run DA batches ahead of the MFMAs while the MFMAs read other
// LDS slots; the waits that make a slot readable are the explicit ones at the
// top of each batch.
// Rows without an A block are zeroed when the operand is read from LDS; a
// column whose B strip is absent has no active slot and issues no MFMA.
// ---------------------------------------------------------------------------
// Tile scheduling of the product kernels.  XCD x owns the contiguous tile
// range [ntiles x / 8, ntiles (x + 1) / 8) (workgroups are dealt to the 8 XCDs
// round robin, so concurrent tiles of one XCD share operands through its L2)
// and its workgroups take those tiles in order from the counter queue[x]
// (zero at launch).  A workgroup whose XCD has run out takes tiles from the
// other XCDs' counters (XCD x+1, x+2, ...), so the launch ends when all tiles
// are taken; -1 then.  Called by one thread; `victim` (0 .. 8) is that
// thread's position in the XCD order and only grows.
// ---------------------------------------------------------------------------
__device__ __forceinline__ i64 next_tile(unsigned long long* queue, i64 ntiles, int xcd, int& victim) {
  while (victim < 8) {
    const int x = (xcd + victim) & 7;
    const i64 b = ntiles * x / 8, e = ntiles * (x + 1) / 8;
    const i64 t = b + (i64)atomicAdd(&queue[x], 1ull);
    if (t < e) return t;
    ++victim;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Steps per staged batch and copy lookahead (LDS per workgroup: (DA+1) SB
// steps of operands and (DA+2) SB records).
#ifndef LSDM_GSB_F32
#define LSDM_GSB_F32 4
#endif
#ifndef LSDM_GSB_F64
#define LSDM_GSB_F64 2
#endif
#ifndef LSDM_GDA
#define LSDM_GDA 1
#endif
template <class T> struct GCfg;
template <> struct GCfg<float> { static constexpr int SB = LSDM_GSB_F32; };
template <> struct GCfg<double> { static constexpr int SB = LSDM_GSB_F64; };

typedef int i4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// 16 bytes per lane from global memory to LDS at dst + 16 * lane
__device__ __forceinline__ void copy16(const void* src, void* dst) {
  __builtin_amdgcn_global_load_lds((glb_void_t*)src, (lds_void_t*)dst, 16, 0, 0);
}
// s_waitcnt immediates (gfx9 encoding): vmcnt(n) alone, lgkmcnt(0) alone
constexpr int waitcnt_vm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x70 | 0xF00; }
constexpr int WAIT_LGKM0 = 15 | (3 << 14) | 0x70;

template <class T>
struct GLayout {
  static constexpr int SB = GCfg<T>::SB;
  static constexpr int DA = LSDM_GDA;
  static constexpr int NDS = DA + 1;          // operand slots
  static constexpr int NRS = DA + 2;          // record slots
  static constexpr int AV = GROWS * 16;       // A values of one step
  static constexpr int BV = GJ * 64;          // B values of one step
  static constexpr int SV = AV + BV;
  static constexpr int VPL = 16 / (int)sizeof(T);
  static constexpr int PV = 64 * VPL;         // values of one 1 KB piece
  static constexpr int PPS = SV / PV;         // pieces per step
  static constexpr int NPW = SB * PPS / GQ;   // pieces per wavefront and batch
  static constexpr int RW = 32;               // dwords per record
  static constexpr int RLANES = SB * RW / 4;  // lanes of the record copy
  static_assert(AV % PV == 0 && BV % PV == 0 && (SB * PPS) % GQ == 0 && RLANES <= 64 && DA >= 1, "staging");
};

// LDS reads of the batch function are written out with their wait in the
// same asm statement: the compiler, which cannot tell them apart from the
// copies still in flight into other slots, would otherwise wait for every
// copy before each read.  Their outputs are early-clobber: a statement issues
// several reads, so no output may share a register with an address input.
typedef __attribute__((address_space(3))) char lds_char;
__device__ __forceinline__ uint32_t lds_off(const void* p) { return (uint32_t)(uintptr_t)(const lds_char*)p; }
// A operand at a, the 8 B operands at b + 64 j values
template <class T>
__device__ __forceinline__ void lds_operands(uint32_t a, uint32_t b, T& av, T (&bv)[GJ]);
template <>
__device__ __forceinline__ void lds_operands<float>(uint32_t a, uint32_t b, float& av, float (&bv)[GJ]) {
  static_assert(GJ == 8, "operand read layout");
  asm volatile(
      "ds_read_b32 %0, %9\n\t"
      "ds_read_b32 %1, %10\n\t"
      "ds_read_b32 %2, %10 offset:256\n\t"
      "ds_read_b32 %3, %10 offset:512\n\t"
      "ds_read_b32 %4, %10 offset:768\n\t"
      "ds_read_b32 %5, %10 offset:1024\n\t"
      "ds_read_b32 %6, %10 offset:1280\n\t"
      "ds_read_b32 %7, %10 offset:1536\n\t"
      "ds_read_b32 %8, %10 offset:1792\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(av), "=&v"(bv[0]), "=&v"(bv[1]), "=&v"(bv[2]), "=&v"(bv[3]), "=&v"(bv[4]), "=&v"(bv[5]),
        "=&v"(bv[6]), "=&v"(bv[7])
      : "v"(a), "v"(b));
}
template <>
__device__ __forceinline__ void lds_operands<double>(uint32_t a, uint32_t b, double& av, double (&bv)[GJ]) {
  static_assert(GJ == 8, "operand read layout");
  asm volatile(
      "ds_read_b64 %0, %9\n\t"
      "ds_read_b64 %1, %10\n\t"
      "ds_read_b64 %2, %10 offset:512\n\t"
      "ds_read_b64 %3, %10 offset:1024\n\t"
      "ds_read_b64 %4, %10 offset:1536\n\t"
      "ds_read_b64 %5, %10 offset:2048\n\t"
      "ds_read_b64 %6, %10 offset:2560\n\t"
      "ds_read_b64 %7, %10 offset:3072\n\t"
      "ds_read_b64 %8, %10 offset:3584\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(av), "=&v"(bv[0]), "=&v"(bv[1]), "=&v"(bv[2]), "=&v"(bv[3]), "=&v"(bv[4]), "=&v"(bv[5]),
        "=&v"(bv[6]), "=&v"(bv[7])
      : "v"(a), "v"(b));
}

// Exchange across the 4 lanes of a quad (DPP quad_perm): lane c gets v of
// lane perm[c].
template <int CTRL>
__device__ __forceinline__ float quad_perm(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
// 4x4 transpose held by the 4 lanes of a quad: on entry lane c (c = lane & 3)
// holds column c (a[r] = M[r][c]), on exit row c (a[x] = M[c][x]).  Two
// butterfly rounds: lanes c and c^2 swap the off-diagonal 2x2 halves, then
// lanes c and c^1 swap the off-diagonal elements of each 2x2 block.  Every
// lane of the quad must execute it.
__device__ __forceinline__ void quad_transpose(float (&a)[4], int c) {
  const bool h = (c & 2) != 0;
  float s0 = h ? a[0] : a[2], s1 = h ? a[1] : a[3];
  float r0 = quad_perm<0x4E>(s0), r1 = quad_perm<0x4E>(s1);    // lanes [2, 3, 0, 1]
  if (h) { a[0] = r0; a[1] = r1; } else { a[2] = r0; a[3] = r1; }
  const bool odd = (c & 1) != 0;
  s0 = odd ? a[0] : a[1];
  s1 = odd ? a[2] : a[3];
  r0 = quad_perm<0xB1>(s0);                                     // lanes [1, 0, 3, 2]
  r1 = quad_perm<0xB1>(s1);
  if (odd) { a[0] = r0; a[2] = r1; } else { a[1] = r0; a[3] = r1; }
}

// One batch of a group tile: copies for later batches, then the MFMAs of
// this one (see k_gprod).  ring: the workgroup's LDS ring; slot arguments are
// byte offsets into it.
template <class T, bool TA>
__device__ __forceinline__ void gbatch(char* ring, int rec_cur, int op_cur, int rec_addr, int op_dst, int rec_dst,
                                       const char* rec_src, bool do_rec, bool do_ops, int nv,
                                       const T* __restrict__ A, const T* __restrict__ B, int na_blk, int nb_str,
                                       typename Mma16<T>::acc_t (&acc)[GJ], int lane, int wave, int a_off, int b_off,
                                       int abit) {
  typedef GLayout<T> L;
  const uint32_t base = lds_off(ring);
  static_assert(L::NPW == 3, "record field reads below");
  // the operand indices of this wavefront's pieces (records of batch q+DA)
  // and the slot masks / row bits of batch q (lane r < SB: mask of step r,
  // lane SB + r: row bits of step r), all read in one statement
  int fa[L::NPW];
#pragma unroll
  for (int i = 0; i < L::NPW; ++i) {
    const int p = L::NPW * wave + i;
    const int r = p / L::PPS, part = p % L::PPS;
    const int off = part * L::PV + lane * L::VPL;
    const int field = part * L::PV < L::AV ? (off >> 4) : GROWS + ((off - L::AV) >> 6);
    fa[i] = base + rec_addr + 4 * (r * L::RW + field);
  }
  const int mfield = lane < L::SB ? lane * L::RW + GROWS + GJ + wave : (lane - L::SB) * L::RW + GROWS + GJ + GQ;
  const uint32_t ma = base + rec_cur + 4 * (lane < 2 * L::SB ? mfield : 0);
  int idx[L::NPW], mr;
  asm volatile(
      "ds_read_b32 %0, %4\n\t"
      "ds_read_b32 %1, %5\n\t"
      "ds_read_b32 %2, %6\n\t"
      "ds_read_b32 %3, %7\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(idx[0]), "=&v"(idx[1]), "=&v"(idx[2]), "=&v"(mr)
      : "v"(fa[0]), "v"(fa[1]), "v"(fa[2]), "v"(ma));
  // lanes r < SB: the column quads of step r with any active slot of this
  // wavefront (zero past the tile's end); lanes SB + r: row bits of step r
  {
    const uint32_t m = (uint32_t)mr;
    const uint32_t cm = (m | (m >> GJ) | (m >> (2 * GJ)) | (m >> (3 * GJ))) & ((1u << GJ) - 1u);
    mr = lane < L::SB ? (lane < nv ? (int)cm : 0) : mr;
  }
  if (do_rec && wave == 0 && lane < L::RLANES) copy16(rec_src + 16 * lane, ring + rec_dst);
  if (do_ops) {
#pragma unroll
    for (int i = 0; i < L::NPW; ++i) {
      const int p = L::NPW * wave + i;
      const int r = p / L::PPS, part = p % L::PPS;
      const int off = part * L::PV + lane * L::VPL;
      // absent operands (-1) read block 0; indices are clamped to the arrays
      const T* src = part * L::PV < L::AV ? A + (i64)min(max(idx[i], 0), na_blk - 1) * 16 + (off & 15)
                                          : B + (i64)min(max(idx[i], 0), nb_str - 1) * 64 + ((off - L::AV) & 63);
      copy16(src, ring + op_dst + (r * L::SV + part * L::PV) * (int)sizeof(T));
    }
  }
  if (nv <= 0) return;
#pragma unroll
  for (int r = 0; r < L::SB; ++r) {
    const uint32_t mask = (uint32_t)__builtin_amdgcn_readlane(mr, r);
    if (mask == 0u) continue;
    const uint32_t rows = (uint32_t)__builtin_amdgcn_readlane(mr, L::SB + r);
    const uint32_t sA = base + op_cur + r * L::SV * (int)sizeof(T);
    T av, bv[GJ];
    lds_operands<T>(sA + a_off * (int)sizeof(T), sA + (L::AV + b_off) * (int)sizeof(T), av, bv);
    av = ((rows >> abit) & 1u) ? av : (T)0;
#pragma unroll
    for (int j = 0; j < GJ; ++j)
      if (mask & (1u << j)) acc[j] = Mma16<T>::mma(av, bv[j], acc[j]);
  }
}

// Occupancy: the FP32 instance fits 6 workgroups per CU (LDS 26.8 KB, at most
// 80 VGPRs), which measured faster than 5 with deeper staging; the FP64
// instance is bound by its accumulators to 4.
template <class T, bool TA>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 4))) k_gprod(const GTile* __restrict__ tiles, i64 ntiles,
                                               const GStep* __restrict__ steps, const T* __restrict__ A,
                                               const T* __restrict__ B, T* __restrict__ C,
                                               const uint8_t* __restrict__ cmask, T alpha, T beta, int na_blk,
                                               int nb_str, unsigned long long* __restrict__ queue,
                                               const T* __restrict__ Cin, const i64* __restrict__ cmap,
                                               const i32* __restrict__ mirw) {
  typedef typename Mma16<T>::acc_t acc_t;
  typedef GLayout<T> L;
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int SB = L::SB, DA = L::DA;
  // LDS ring: NDS operand slots, then NRS record slots
  constexpr int DSLOT = SB * L::SV * (int)sizeof(T), RSLOT = SB * L::RW * 4;
  __shared__ __attribute__((aligned(16))) char ring[L::NDS * DSLOT + L::NRS * RSLOT];
  auto dslot = [&](int x) { return x * DSLOT; };
  auto rslot = [&](int x) { return L::NDS * DSLOT + x * RSLOT; };
  // output strips of each wavefront's 4 x GJ slots and their block masks
  __shared__ int cstr[GQ][4 * GJ];
  __shared__ uint8_t cmsk[GQ][4 * GJ];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int arow = lane & 15, ai = arow >> 2, ar = arow & 3, kk = lane >> 4;
  const int a_off = (4 * wave + ai) * 16 + (TA ? (kk * 4 + ar) : (ar * 4 + kk));
  const int b_off = ((lane & 15) >> 2) * 16 + kk * 4 + (lane & 3);
  const int abit = 4 * wave + ai;
  // tiles: see next_tile
  const int xcd = (int)(blockIdx.x & 7);
  int victim = 0;
  const char* recs = reinterpret_cast<const char*>(steps);
  __shared__ i64 t_next;

  for (;;) {
    if (threadIdx.x == 0) t_next = next_tile(queue, ntiles, xcd, victim);
    __syncthreads();
    const i64 t = t_next;
    if (t < 0) break;
    const GTile* tp = tiles + uniform64(t);
    const i64 s0 = tp->step0;
    const int ns = tp->nsteps;
    acc_t acc[GJ];
#pragma unroll
    for (int q = 0; q < GJ; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[q][e] = (T)0;
    const int nb = (ns + SB - 1) / SB;
    auto rec_src = [&](int q) { return recs + (s0 + (i64)SB * q) * (i64)sizeof(GStep); };
    // prologue: this wavefront's output strips and masks, records of the
    // first DA+1 batches (every copy complete before the loop)
    const i32 my_cs = lane < 4 * GJ ? tp->cstrip[4 * GJ * wave + lane] : -1;
    if (wave == 0 && lane < L::RLANES)
      for (int q = 0; q <= DA && q < nb; ++q) copy16(rec_src(q) + 16 * lane, ring + rslot(q));
    const int mk = my_cs >= 0 ? (int)cmask[my_cs] : 0;
    if (lane < 4 * GJ) {
      cstr[wave][lane] = my_cs;
      cmsk[wave][lane] = (uint8_t)mk;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // batch q runs the MFMAs of q (q >= 0) and copies operands q+DA and
    // records q+DA+1; batches -DA .. -1 only copy
    // slot numbers of batch q: operands q % NDS, records q % NRS (running)
    int ds0 = ((-DA) % L::NDS + L::NDS) % L::NDS, rs0 = ((-DA) % L::NRS + L::NRS) % L::NRS;
    for (int q = -DA; q < nb; ++q) {
      // this wavefront's copies of operands q and records q+DA are complete
      // (copies complete in issue order; the NPW copies of operands q+DA-1,
      // issued last in batch q-1, may remain if batch q-1 issued them)
      asm volatile("" ::: "memory");
      if (DA >= 2 && q > -DA && q - 1 + DA < nb)
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(L::NPW));
      else
        __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      const int ds1 = ds0 + DA >= L::NDS ? ds0 + DA - L::NDS : ds0 + DA;
      const int rs1 = rs0 + DA >= L::NRS ? rs0 + DA - L::NRS : rs0 + DA;
      const int rs2 = rs1 + 1 >= L::NRS ? rs1 + 1 - L::NRS : rs1 + 1;
      gbatch<T, TA>(ring, rslot(rs0), dslot(ds0), rslot(rs1), dslot(ds1), rslot(rs2),
                    rec_src(q + DA + 1), q + DA + 1 < nb && q + DA + 1 > DA, q + DA < nb,
                    q >= 0 ? ns - SB * q : 0, A, B, na_blk, nb_str, acc, lane, wave, a_off, b_off, abit);
      ds0 = ds0 + 1 == L::NDS ? 0 : ds0 + 1;
      rs0 = rs0 + 1 == L::NRS ? 0 : rs0 + 1;
    }
    // epilogue: lane l, register v holds D[row][col]; f32 row = 4 (l/16) + v,
    // f64 row = 4 v + l/16; col = l % 16 (block t = col / 4, c = col % 4)
    {
      const int col = lane & 15, tb = col >> 2, cc = col & 3;
      // the beta term may come from another pattern's strips (cmap: C strip
      // -> Cin strip), masked to C's blocks; a column quad's map entries are
      // read together before its stores
      // a half-output product of a symmetric result (mirw non-null, no beta
      // term) also writes the dropped half: word w of the block (d_mirw of the
      // pattern) gives its mirror block ((w >> 1) - 1) and whether the block
      // itself is written (w & 1); the mirror's row cc is this block's column cc
      if constexpr (!F64) {
        // FP32: the lane's column (rows 0..3 of block tb) becomes row cc by a
        // quad transpose, written 16 bytes per lane (a strip per 16 lanes)
        const int i = lane >> 4;
#pragma unroll
        for (int j = 0; j < GJ; ++j) {
          const int cs = cstr[wave][GJ * i + j];
          const int mw = (mirw && cs >= 0) ? mirw[4 * (i64)cs + tb] : 1;
          const bool in = cs >= 0 && ((cmsk[wave][GJ * i + j] >> tb) & 1);
          float o[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) o[v] = in ? (float)alpha * (float)acc[j][v] : 0.f;
          if (mw >> 1)
            *reinterpret_cast<float4*>(reinterpret_cast<float*>(C) + (i64)((mw >> 1) - 1) * 16 + cc * 4) =
                make_float4(o[0], o[1], o[2], o[3]);
          quad_transpose(o, cc);
          if (cs >= 0 && (mw & 1)) {
            float4* dst = reinterpret_cast<float4*>(reinterpret_cast<float*>(C) + (i64)cs * 64 + tb * 16 + cc * 4);
            if (cmap) {
              if (in) {
#pragma clang fp contract(off)
                const float4 y = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(Cin) +
                                                                   cmap[cs] * 64 + tb * 16 + cc * 4);
                o[0] += (float)beta * y.x;
                o[1] += (float)beta * y.y;
                o[2] += (float)beta * y.z;
                o[3] += (float)beta * y.w;
              }
            } else if (beta != (T)0) {
              const float4 c = *dst;
              o[0] += (float)beta * c.x;
              o[1] += (float)beta * c.y;
              o[2] += (float)beta * c.z;
              o[3] += (float)beta * c.w;
            }
            *dst = make_float4(o[0], o[1], o[2], o[3]);
          }
        }
      } else {
#pragma unroll
      for (int j = 0; j < GJ; ++j) {
        int mv[4] = {-1, -1, -1, -1};
        if (cmap) {
#pragma unroll
          for (int v = 0; v < (F64 ? 4 : 1); ++v) {
            const int cs = cstr[wave][GJ * (F64 ? v : (lane >> 4)) + j];
            mv[v] = cs >= 0 ? (int)cmap[cs] : -1;
          }
          if (!F64) mv[1] = mv[2] = mv[3] = mv[0];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = F64 ? v : (lane >> 4);
          const int rr = F64 ? (lane >> 4) : v;
          const int2 ci = int2{cstr[wave][GJ * i + j], (int)cmsk[wave][GJ * i + j]};
          if (ci.x < 0) continue;
          const i64 idx = (i64)ci.x * 64 + tb * 16 + rr * 4 + cc;
          const bool in = (ci.y >> tb) & 1;
          T o = in ? alpha * acc[j][v] : (T)0;
          if (mirw) {
            const int w = mirw[4 * (i64)ci.x + tb];
            if (w >> 1) C[(i64)((w >> 1) - 1) * 16 + cc * 4 + rr] = o;   // element (cc, rr) of the mirror
            if (!(w & 1)) continue;
          }
          if (cmap) {
            // rounded as a separate scaled copy of Cin would be (no fused
            // multiply-add), so the result does not depend on the route
#pragma clang fp contract(off)
            if (in) o += beta * Cin[(i64)mv[v] * 64 + (idx & 63)];
          } else if (beta != (T)0) {
            o += beta * C[idx];
          }
          C[idx] = o;
        }
      }
      }
    }
    // the next tile's prologue rewrites record slots and the slot table
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// BF16 group-tile product: register staging of bf16 operands (8 bytes per
// lane per piece) and gfx950's v_mfma_f32_16x16x32_bf16, one instruction per
// active column quad covering a batch's 8 steps: lane l holds
// A[l%16][8g..8g+7] and B[8g..8g+7][l%16] for g = l/16, the k values of steps
// 2g and 2g+1, i.e. one row of A_{r,k} (a column of X_{k,r} for a transposed
// A, from the column-major copy) and one column of a B block (column-major
// copy) of each of the two steps; D[4(l/16)+v][l%16] as for FP32.  A step's
// half is zeroed where the step lies past the tile's end, its row has no A
// block, or (for B) its column quad has no B strip.  The epilogue can also
// write bf16 copies of the result (row-major and block-transposed) for the
// products that take it as an operand, rounded from the FP32 value.
// ---------------------------------------------------------------------------
typedef int i2v __attribute__((ext_vector_type(2)));


template <bool TA>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_gprod_bf16(const GTile* __restrict__ tiles, i64 ntiles,
                                                    const GStep* __restrict__ steps,
                                                    const unsigned short* __restrict__ A,
                                                    const unsigned short* __restrict__ B, float* __restrict__ C,
                                                    unsigned short* __restrict__ outR, unsigned short* __restrict__ outC,
                                                    const uint8_t* __restrict__ cmask, float alpha, float beta,
                                                    unsigned long long* __restrict__ queue, const i64* __restrict__ cmir,
                                                    const i32* __restrict__ csquad, const i32* __restrict__ csimg,
                                                    const uint8_t* __restrict__ cneed, const float* __restrict__ Cin,
                                                    const i64* __restrict__ cmap) {
  constexpr int SB = 8;                 // steps per batch: one MFMA of K = 32 per column quad
  constexpr int AV = GROWS * 16;
  constexpr int BV = GJ * 64;
  constexpr int SV = AV + BV;
  constexpr int VPL = 4;                // bf16 values per lane of one piece (8 bytes)
  constexpr int PV = 64 * VPL;
  constexpr int PPS = SV / PV;
  constexpr int SPW = SB / GQ;
  constexpr int NPW = SPW * PPS;
  constexpr int RW = 32;
  constexpr int RLANES = SB * RW / 4;
  static_assert(AV % PV == 0 && BV % PV == 0 && SB % GQ == 0 && SB == 2 * GQ && RLANES <= 64, "staging layout");
  __shared__ __attribute__((aligned(16))) unsigned short dbuf[2][SB * SV];
  __shared__ __attribute__((aligned(16))) int rbuf[3][SB * RW];
  __shared__ int cstr[GQ][4 * GJ];
  __shared__ uint8_t cmsk[GQ][4 * GJ];
  // symmetric results: mirror block (value offset / 16) of each slot's 4
  // blocks and which of block / mirror the epilogue writes (bits tb, 4 + tb)
  __shared__ int4 cmb[GQ][4 * GJ];
  __shared__ uint8_t cwr[GQ][4 * GJ];
  __shared__ int cmp[GQ][4 * GJ];   // cmap of each slot's strip (-1: none)

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int arow = lane & 15, ai = arow >> 2, ar = arow & 3, ks = lane >> 4;
  const int a_off = (4 * wave + ai) * 16 + ar * 4;
  const int b_off = ((lane & 15) >> 2) * 16 + (lane & 3) * 4;
  const int abit = 4 * wave + ai;
  constexpr uint32_t COL = 1u | (1u << GJ) | (1u << (2 * GJ)) | (1u << (3 * GJ));
  // tiles: see next_tile (per-XCD counters, then the other XCDs' tiles)
  const int xcd = (int)(blockIdx.x & 7);
  int victim = 0;
  const i4v* recs = reinterpret_cast<const i4v*>(steps);
  __shared__ i64 t_next;

  for (;;) {
    if (threadIdx.x == 0) t_next = next_tile(queue, ntiles, xcd, victim);
    __syncthreads();
    const i64 t = t_next;
    if (t < 0) break;
    const GTile* tp = tiles + uniform64(t);
    const i64 s0 = tp->step0;
    const int ns = tp->nsteps;
    f4 acc[GJ];
#pragma unroll
    for (int q = 0; q < GJ; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[q][e] = 0.f;
    const int nb = (ns + SB - 1) / SB;
    auto load_records = [&](int q) -> i4v {
      i4v v = {0, 0, 0, 0};
      if (wave == 0 && lane < RLANES) v = recs[(s0 + (i64)SB * q) * (RW / 4) + lane];
      return v;
    };
    auto store_records = [&](const i4v& v, int slot) {
      if (wave == 0 && lane < RLANES) *reinterpret_cast<i4v*>(&rbuf[slot][4 * lane]) = v;
    };
    auto load_operands = [&](int rslot, i2v (&d)[NPW]) {
      int idx[NPW];
#pragma unroll
      for (int i = 0; i < NPW; ++i) {
        const int r = SPW * wave + i / PPS, part = i % PPS;
        const int off = part * PV + lane * VPL;
        idx[i] = part * PV < AV ? rbuf[rslot][r * RW + (off >> 4)] : rbuf[rslot][r * RW + GROWS + ((off - AV) >> 6)];
      }
#pragma unroll
      for (int i = 0; i < NPW; ++i) {
        const int part = i % PPS;
        const int off = part * PV + lane * VPL;
        const unsigned short* src = part * PV < AV ? A + (i64)max(idx[i], 0) * 16 + (off & 15)
                                                   : B + (i64)max(idx[i], 0) * 64 + ((off - AV) & 63);
        d[i] = *reinterpret_cast<const i2v*>(src);
      }
    };
    auto store_operands = [&](const i2v (&d)[NPW], int dslot) {
#pragma unroll
      for (int i = 0; i < NPW; ++i) {
        const int r = SPW * wave + i / PPS, part = i % PPS;
        *reinterpret_cast<i2v*>(&dbuf[dslot][r * SV + part * PV + lane * VPL]) = d[i];
      }
    };
    const i32 my_cs = lane < 4 * GJ ? tp->cstrip[4 * GJ * wave + lane] : -1;
    if (nb > 0) {
      {
        const i4v r0 = load_records(0);
        const i4v r1 = nb > 1 ? load_records(1) : i4v{0, 0, 0, 0};
        store_records(r0, 0);
        store_records(r1, 1);
      }
      __syncthreads();
      {
        i2v d[NPW];
        load_operands(0, d);
        // block mask, and bit 4: the FP32 result is written on this strip
        const int mk = my_cs >= 0 ? (int)cmask[my_cs] | ((!cneed || cneed[my_cs]) ? 16 : 0) : 0;
        const int mp = (cmap && my_cs >= 0) ? (int)cmap[my_cs] : -1;
        store_operands(d, 0);
        if (lane < 4 * GJ) {
          cstr[wave][lane] = my_cs;
          cmsk[wave][lane] = (uint8_t)mk;
          cmp[wave][lane] = mp;
        }
      }
    } else if (lane < 4 * GJ) {
      cstr[wave][lane] = my_cs;
      cmsk[wave][lane] = (uint8_t)(my_cs >= 0 ? (int)cmask[my_cs] | ((!cneed || cneed[my_cs]) ? 16 : 0) : 0);
      cmp[wave][lane] = (cmap && my_cs >= 0) ? (int)cmap[my_cs] : -1;
    }
    // mirror writes of this wavefront's slots (lane = slot GJ i + jq, row i of
    // its quad), loaded now and kept in registers until the epilogue.  In the
    // row's own quad at image 0 the blocks below the diagonal are written only
    // as mirrors of the blocks above it.
    int4 my_mb = int4{-1, -1, -1, -1};
    int my_wr = 0x0f;
    if (cmir && lane < 4 * GJ && my_cs >= 0) {
      const i32 prow = GROWS * tp->group + 4 * wave + lane / GJ, cq = csquad[my_cs];
      const bool own = cq == (prow >> 2) && csimg[my_cs] == IMG0;
      int mb[4];
      my_wr = 0;
#pragma unroll
      for (int tb = 0; tb < 4; ++tb) {
        const i32 qcol = 4 * cq + tb;
        const bool self = !(own && qcol < prow), mir = !(own && qcol <= prow);
        const i64 m = mir ? cmir[4 * (i64)my_cs + tb] : -1;
        mb[tb] = m >= 0 ? (int)(m >> 4) : -1;
        my_wr |= (self ? 1 : 0) << tb;
      }
      my_mb = int4{mb[0], mb[1], mb[2], mb[3]};
    }
    for (int q = 0; q < nb; ++q) {
      __syncthreads();
      const bool more_r = q + 2 < nb, more_d = q + 1 < nb;
      i4v rn = {0, 0, 0, 0};
      i2v dn[NPW];
      if (more_r) rn = load_records(q + 2);
      if (more_d) load_operands((q + 1) % 3, dn);
      const int rs = q % 3, ds = q & 1;
      const int nv = ns - SB * q;
      {
        // one v_mfma_f32_16x16x32_bf16 per active column quad covers the
        // batch's 8 steps: lane group ks holds steps 2 ks and 2 ks + 1 (8
        // consecutive k values), each half zeroed on its own where its step
        // lies past the tile's end, its row has no A block or its column no
        // B strip
        const int rl0 = 2 * ks, rl1 = rl0 + 1;
        const int* rec0 = &rbuf[rs][rl0 * RW];
        const int* rec1 = &rbuf[rs][rl1 * RW];
        const bool v0 = rl0 < nv, v1 = rl1 < nv;
        const uint32_t m_l = (v0 ? (uint32_t)rec0[GROWS + GJ + wave] : 0u) | (v1 ? (uint32_t)rec1[GROWS + GJ + wave] : 0u);
        const uint32_t colany = (uint32_t)__builtin_amdgcn_readlane((int)m_l, 0) |
                                (uint32_t)__builtin_amdgcn_readlane((int)m_l, 16) |
                                (uint32_t)__builtin_amdgcn_readlane((int)m_l, 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int)m_l, 48);
        if (colany != 0u) {
          const uint32_t rows0 = (uint32_t)rec0[GROWS + GJ + GQ], rows1 = (uint32_t)rec1[GROWS + GJ + GQ];
          const uint32_t bc0 = (uint32_t)rec0[GROWS + GJ + GQ + 1], bc1 = (uint32_t)rec1[GROWS + GJ + GQ + 1];
          const unsigned short* sS0 = &dbuf[ds][rl0 * SV];
          const unsigned short* sS1 = &dbuf[ds][rl1 * SV];
          s4 a0 = *reinterpret_cast<const s4*>(sS0 + a_off);
          s4 a1 = *reinterpret_cast<const s4*>(sS1 + a_off);
          if (!(v0 && ((rows0 >> abit) & 1u))) a0 = s4{0, 0, 0, 0};
          if (!(v1 && ((rows1 >> abit) & 1u))) a1 = s4{0, 0, 0, 0};
          const bf8 av = __builtin_bit_cast(bf8, __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7));
#pragma unroll
          for (int j = 0; j < GJ; ++j) {
            if (!((colany >> j) & COL)) continue;
            s4 b0 = *reinterpret_cast<const s4*>(sS0 + AV + j * 64 + b_off);
            s4 b1 = *reinterpret_cast<const s4*>(sS1 + AV + j * 64 + b_off);
            if (!((bc0 >> j) & 1u)) b0 = s4{0, 0, 0, 0};
            if (!((bc1 >> j) & 1u)) b1 = s4{0, 0, 0, 0};
            const bf8 bv = __builtin_bit_cast(bf8, __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7));
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[j], 0, 0, 0);
          }
        }
      }
      if (more_d) store_operands(dn, (q + 1) & 1);
      if (more_r) store_records(rn, (q + 2) % 3);
    }
    {
      // lane l holds rows 0..3 of column cc of block tb in row i of its row
      // quad; the bf16 copies are written 8 bytes per lane: the
      // block-transposed copy (outC) takes the lane's column as is, the
      // row-major copy (outR) and the mirror block of a symmetric result take
      // row cc after a transpose across the lane's quad
      const int col = lane & 15, tb = col >> 2, cc = col & 3, i = lane >> 4;
      if (cmir) {
        if (lane < 4 * GJ) {
          cmb[wave][lane] = my_mb;
          cwr[wave][lane] = (uint8_t)my_wr;
        }
        __builtin_amdgcn_wave_barrier();
      }
#pragma unroll
      for (int j = 0; j < GJ; ++j) {
        const int cs = cstr[wave][GJ * i + j];
        const int mk = cmsk[wave][GJ * i + j];
        const bool in = cs >= 0 && ((mk >> tb) & 1);
        float o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = in ? alpha * acc[j][v] : 0.f;
        // a symmetric result (cmir non-null, half plan) also gets its dropped
        // half: the block-transposed copy of the mirror block (q, p, -n) is the
        // row-major copy of this block (slot tables above)
        bool self = true;
        i64 mirror = -1;
        if (cmir && cs >= 0) {
          const int4 mbv = cmb[wave][GJ * i + j];
          self = (cwr[wave][GJ * i + j] >> tb) & 1;
          const int mbi = tb == 0 ? mbv.x : tb == 1 ? mbv.y : tb == 2 ? mbv.z : mbv.w;
          mirror = mbi >= 0 ? (i64)mbi * 16 : -1;
        }
        // copies rounded from the FP32 result as a separate conversion pass
        // would; without a beta term the block-transposed copy is the lane's
        // column as it stands
        const bool plain = beta == 0.f && !cmap;
        if (outC && plain && cs >= 0 && self)
          *reinterpret_cast<ushort4*>(outC + (i64)cs * 64 + tb * 16 + cc * 4) =
              make_ushort4(bf16_rne(o[0]), bf16_rne(o[1]), bf16_rne(o[2]), bf16_rne(o[3]));
        quad_transpose(o, cc);               // o[x] = row cc, column x
        if (cs >= 0) {
          const i64 rb = (i64)cs * 64 + tb * 16 + cc * 4;
          if (cmap) {   // the beta term from another pattern's strips (see k_gprod)
            if (in) {
#pragma clang fp contract(off)
              const float4 y = *reinterpret_cast<const float4*>(Cin + (i64)cmp[wave][GJ * i + j] * 64 + tb * 16 + cc * 4);
              o[0] += beta * y.x;
              o[1] += beta * y.y;
              o[2] += beta * y.z;
              o[3] += beta * y.w;
            }
          } else if (beta != 0.f) {
            const float4 c = *reinterpret_cast<const float4*>(C + rb);
            o[0] += beta * c.x;
            o[1] += beta * c.y;
            o[2] += beta * c.z;
            o[3] += beta * c.w;
          }
          if (C && ((mk >> 4) & 1)) *reinterpret_cast<float4*>(C + rb) = make_float4(o[0], o[1], o[2], o[3]);
          const ushort4 row = make_ushort4(bf16_rne(o[0]), bf16_rne(o[1]), bf16_rne(o[2]), bf16_rne(o[3]));
          if (outR) *reinterpret_cast<ushort4*>(outR + rb) = row;
          if (mirror >= 0) *reinterpret_cast<ushort4*>(outC + mirror + cc * 4) = row;
        }
        if (outC && !plain) {               // back to the column for the block-transposed copy
          quad_transpose(o, cc);
          if (cs >= 0 && self)
            *reinterpret_cast<ushort4*>(outC + (i64)cs * 64 + tb * 16 + cc * 4) =
                make_ushort4(bf16_rne(o[0]), bf16_rne(o[1]), bf16_rne(o[2]), bf16_rne(o[3]));
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Residual mode.  Each operand is split into its on-site part D (atom blocks
// (a, a, 0); with pseudo-atoms, every pair of pseudo-atoms of one atom) and
// the rest R: AB = R_A R_B + D_A B + A D_B - D_A D_B.  R_A R_B runs on the FP32
// product kernel; the other three terms are block-diagonal scalings done here
// in FP64.  The blocks each output block needs are found once per plan (binary
// search in the strip lists) and kept as index maps.
// ---------------------------------------------------------------------------
struct PatDev {
  const i64* sptr;
  const i32* squad;
  const i32* simg;
  const uint8_t* smask;
};

// value offset of block (row, col, img) of a pattern, -1 when outside it
__device__ __forceinline__ i64 block_off(const PatDev& p, i32 row, i32 col, i32 img) {
  const i64 key = skey(col >> 2, img);
  i64 lo = p.sptr[row], hi = p.sptr[row + 1];
  while (lo < hi) {
    const i64 mid = (lo + hi) >> 1;
    if (skey(p.squad[mid], p.simg[mid]) < key) lo = mid + 1; else hi = mid;
  }
  if (lo < p.sptr[row + 1] && skey(p.squad[lo], p.simg[lo]) == key && ((p.smask[lo] >> (col & 3)) & 1))
    return lo * 64 + (col & 3) * 16;
  return -1;
}

// FP64 strips -> FP32 copy with the on-site blocks set to zero
__global__ void k_offsite_f32(const double* __restrict__ in, float* __restrict__ out, const i32* __restrict__ srow,
                              const i32* __restrict__ squad, const i32* __restrict__ simg,
                              const i32* __restrict__ patom, i64 nstrips) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nstrips * 64; g += (i64)gridDim.x * blockDim.x) {
    const i64 st = g >> 6;
    const int t = (int)((g >> 4) & 3);
    const i32 p = srow[st], q = 4 * squad[st] + t;
    const bool onsite = simg[st] == IMG0 && patom[p] >= 0 && patom[p] == patom[q];
    out[g] = onsite ? 0.f : (float)in[g];
  }
}

// op(A)_{p,(x,m)}: A's block (p, x, m), or for a transposed A the transpose
// of A's block (x, p, -m); value offset or -1
template <bool TA>
__device__ __forceinline__ i64 opa_off(const PatDev& A, i32 p, i32 x, i32 m) {
  return TA ? block_off(A, x, p, img_neg(m)) : block_off(A, p, x, m);
}
__device__ __forceinline__ i32 blk_index(i64 off) { return off < 0 ? -1 : (i32)(off >> 4); }

// residual-mode maps of a plan, one thread per output block (see lsdm_plan)
template <bool TA>
__global__ void k_rc_map(PatDev A, PatDev B, PatDev C, const i32* __restrict__ srow, const i32* __restrict__ patom,
                         const i32* __restrict__ pbase, const i32* __restrict__ npseudo, int np, i64 ncstrips,
                         i32* __restrict__ bmap, i32* __restrict__ amap) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < ncstrips * 4; g += (i64)gridDim.x * blockDim.x) {
    const i64 st = g >> 2;
    const int t = (int)(g & 3);
    const i32 p = srow[st], q = 4 * C.squad[st] + t, n = C.simg[st];
    const i32 ap = patom[p], aq = patom[q];
    for (int u = 0; u < np; ++u) {
      i64 b = -1, a = -1;
      if (ap >= 0 && u < npseudo[ap]) b = block_off(B, pbase[ap] + u, q, n);
      if (aq >= 0 && u < npseudo[aq]) a = opa_off<TA>(A, p, pbase[aq] + u, n);
      bmap[g * np + u] = blk_index(b);
      amap[g * np + u] = blk_index(a);
    }
  }
}
template <bool TA>
__global__ void k_rc_onsite(PatDev A, PatDev B, const i32* __restrict__ patom, const i32* __restrict__ pbase,
                            const i32* __restrict__ npseudo, int np, i32 n_pseudo, i32* __restrict__ aon,
                            i32* __restrict__ bon) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < (i64)n_pseudo * np; g += (i64)gridDim.x * blockDim.x) {
    const i32 p = (i32)(g / np);
    const int u = (int)(g % np);
    const i32 ap = patom[p];
    i64 a = -1, b = -1;
    if (ap >= 0 && u < npseudo[ap]) {
      a = opa_off<TA>(A, p, pbase[ap] + u, IMG0);
      b = block_off(B, pbase[ap] + u, p, IMG0);
    }
    aon[g] = blk_index(a);
    bon[g] = blk_index(b);
  }
}

// C = alpha (RR + D_A B + A D_B - D_A D_B) + beta C in FP64, one thread per
// output element (16 per block), the blocks it needs read from the maps; a
// half-output plan (half = 1) skips the strips its mirror fill writes
template <bool TA>
__global__ void k_rc_apply(const uint8_t* __restrict__ cmask, const i32* __restrict__ srow,
                           const i32* __restrict__ csquad, const i32* __restrict__ csimg,
                           const i32* __restrict__ patom, int np, const i32* __restrict__ bmap,
                           const i32* __restrict__ amap, const i32* __restrict__ aon, const i32* __restrict__ bon,
                           const double* __restrict__ A64, const double* __restrict__ B64,
                           const float* __restrict__ RR, double* __restrict__ C64, i64 ncstrips, double alpha,
                           double beta, int half) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < ncstrips * 64; g += (i64)gridDim.x * blockDim.x) {
    const i64 st = g >> 6, blk = g >> 4;
    if (half && !keep_strip(srow[st], csquad[st], csimg[st])) continue;
    const int t = (int)((g >> 4) & 3), e = (int)(g & 15), r = e >> 2, c = e & 3;
    const bool in = (cmask[st] >> t) & 1;
    double acc = 0.0;
    if (in) {
      const i32 p = srow[st], q = 4 * csquad[st] + t, n = csimg[st];
      auto prod = [&](i32 a, i32 b) -> double {
        const double* Ab = A64 + (i64)a * 16;
        const double* Bb = B64 + (i64)b * 16;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) v += (TA ? Ab[k * 4 + r] : Ab[r * 4 + k]) * Bb[k * 4 + c];
        return v;
      };
      for (int u = 0; u < np; ++u) {   // D_A B
        const i32 a = aon[(i64)p * np + u], b = bmap[blk * np + u];
        if (a >= 0 && b >= 0) acc += prod(a, b);
      }
      for (int u = 0; u < np; ++u) {   // A D_B
        const i32 a = amap[blk * np + u], b = bon[(i64)q * np + u];
        if (a >= 0 && b >= 0) acc += prod(a, b);
      }
      if (n == IMG0 && patom[p] >= 0 && patom[p] == patom[q])
        for (int u = 0; u < np; ++u) {   // - D_A D_B (counted in both terms above)
          const i32 a = aon[(i64)p * np + u], b = bon[(i64)q * np + u];
          if (a >= 0 && b >= 0) acc -= prod(a, b);
        }
    }
    double o = in ? alpha * ((double)RR[g] + acc) : 0.0;
    if (beta != 0.0) o += beta * C64[g];
    C64[g] = o;
  }
}

// ---------------------------------------------------------------------------
// K = 3 M|_H - 2 P on H's strips (FP64), masked to H's pattern; an H strip
// outside M's pattern (h2m = -1: beyond the range of LSL) takes M as zero.
// Symmetric results (sym non-null) may hold only their kept half: a block of
// the dropped half (same rule for an H strip and the M strip with the same
// row, quad and image) reads the transpose of its mirror in M and in P, the
// values a mirror fill would have copied there (zero when absent).
// ---------------------------------------------------------------------------
struct KSym {
  const i64* mir_m;    // M's mirror map
  const i64* mir_h;    // H's mirror map (P lives on H's pattern)
  const i32* srow;     // H's strips: row, column quad, image
  const i32* squad;
  const i32* simg;
};

template <class T>
__global__ void k_kassembly(const T* __restrict__ M, const T* __restrict__ P, double* __restrict__ K,
                            const i64* __restrict__ h2m, const uint8_t* __restrict__ hmask, i64 nh, KSym sym) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nh * 64; g += (i64)gridDim.x * blockDim.x) {
    const i64 h = g >> 6;
    const int e = (int)(g & 63), t = e >> 4, r = (e >> 2) & 3, c = e & 3;
    const bool in = (hmask[h] >> t) & 1;
    const i64 m = h2m[h];
    bool dropped = false;
    if (sym.srow) {
      const i32 p = sym.srow[h], q = sym.squad[h], n = sym.simg[h];
      dropped = !keep_strip(p, q, n) || (q == (p >> 2) && n == IMG0 && 4 * q + t < p);
    }
    double mv = 0.0, pv = 0.0;
    if (!dropped) {
      if (m >= 0) mv = (double)M[m * 64 + e];
      if (P) pv = (double)P[g];
    } else {
      const i64 mm = m >= 0 ? sym.mir_m[4 * m + t] : -1;
      const i64 mh = sym.mir_h[4 * h + t];
      if (mm >= 0) mv = (double)M[mm + c * 4 + r];
      if (P && mh >= 0) pv = (double)P[mh + c * 4 + r];
    }
    K[g] = in ? (P ? 3.0 * mv - 2.0 * pv : 3.0 * mv) : 0.0;
  }
}

// out = scale * P_out(in): every strip of `out`'s pattern takes the strip
// map[s] of `in` (a pattern containing out's), masked to out's blocks
template <class T>
__global__ void k_project_strips(const T* __restrict__ in, T* __restrict__ out, const i64* __restrict__ map,
                                 const uint8_t* __restrict__ omask, i64 nout, T scale) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nout * 64; g += (i64)gridDim.x * blockDim.x) {
    const i64 st = g >> 6;
    const int e = (int)(g & 63);
    out[g] = ((omask[st] >> (e >> 4)) & 1) ? scale * in[map[st] * 64 + e] : (T)0;
  }
}

// Mbar += scale * H on the blocks of H inside M's pattern (H's strips mapped
// into M's strips; blocks outside M's, which LSL cannot reach, are skipped,
// so Mbar stays zero off its pattern)
template <class T>
__global__ void k_scatter_h(const T* __restrict__ H, T* __restrict__ Mb, const i64* __restrict__ h2m,
                            const uint8_t* __restrict__ mmask, i64 nh, T scale) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nh * 64; g += (i64)gridDim.x * blockDim.x) {
    const i64 h = g >> 6;
    const int e = (int)(g & 63);
    const i64 m = h2m[h];
    if (m >= 0 && ((mmask[m] >> (e >> 4)) & 1)) Mb[m * 64 + e] += scale * H[g];
  }
}

// ---------------------------------------------------------------------------
// bitwise-reproducible FP64 dot: a fixed grid, each thread sums a fixed
// strided subsequence with Neumaier compensation, then fixed-order trees
// ---------------------------------------------------------------------------
struct Comp {
  double s, c;
};
__device__ __forceinline__ void comp_add(Comp& a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x)) a.c += (a.s - t) + x; else a.c += (x - t) + a.s;
  a.s = t;
}
__device__ __forceinline__ Comp comp_merge(Comp a, Comp b) {
  comp_add(a, b.s);
  a.c += b.c;
  return a;
}

template <class TB>
__global__ void __launch_bounds__(256) k_dot_partial(const double* __restrict__ a, const TB* __restrict__ b, i64 n,
                                                     double* __restrict__ partial) {
  __shared__ double ss[256], sc[256];
  Comp acc{0.0, 0.0};
  for (i64 i = blockIdx.x * 256 + threadIdx.x; i < n; i += (i64)gridDim.x * 256) comp_add(acc, a[i] * (double)b[i]);
  ss[threadIdx.x] = acc.s;
  sc[threadIdx.x] = acc.c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      Comp m = comp_merge(Comp{ss[threadIdx.x], sc[threadIdx.x]}, Comp{ss[threadIdx.x + w], sc[threadIdx.x + w]});
      ss[threadIdx.x] = m.s;
      sc[threadIdx.x] = m.c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = ss[0];
    partial[2 * blockIdx.x + 1] = sc[0];
  }
}

__global__ void __launch_bounds__(256) k_dot_final(const double* __restrict__ partial, int np, double scale,
                                                   double* __restrict__ out) {
  __shared__ double ss[256], sc[256];
  Comp acc{0.0, 0.0};
  for (int i = threadIdx.x; i < np; i += 256) acc = comp_merge(acc, Comp{partial[2 * i], partial[2 * i + 1]});
  ss[threadIdx.x] = acc.s;
  sc[threadIdx.x] = acc.c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      Comp m = comp_merge(Comp{ss[threadIdx.x], sc[threadIdx.x]}, Comp{ss[threadIdx.x + w], sc[threadIdx.x + w]});
      ss[threadIdx.x] = m.s;
      sc[threadIdx.x] = m.c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = scale * (ss[0] + sc[0]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_for(i64 n, int per = 256) {
  i64 g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

template <class T>
void fill(T* p, i64 n, T v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
}
template void fill<double>(double*, i64, double, hipStream_t);
template void fill<float>(float*, i64, float, hipStream_t);
template void fill<unsigned short>(unsigned short*, i64, unsigned short, hipStream_t);

template <class T>
void user_to_strip(const lsdm_pattern* p, const double* user, T* strip, double scale, hipStream_t st) {
  ensure_maps(const_cast<lsdm_pattern*>(p));
  if (p->n_sub == 0) return;
  hipLaunchKernelGGL(k_user_to_strip<T>, dim3(grid_for(p->n_sub * 4)), dim3(256), 0, st, user, strip,
                     p->d_sub_user.as<i64>(), p->d_sub_strip.as<i64>(), p->d_sub_shape.as<i32>(), p->n_sub, scale);
}
template void user_to_strip<double>(const lsdm_pattern*, const double*, double*, double, hipStream_t);
template void user_to_strip<float>(const lsdm_pattern*, const double*, float*, double, hipStream_t);

template <class T>
void strip_to_user(const lsdm_pattern* p, const T* strip, double* user, hipStream_t st) {
  ensure_maps(const_cast<lsdm_pattern*>(p));
  if (p->n_sub == 0) return;
  hipLaunchKernelGGL(k_strip_to_user<T>, dim3(grid_for(p->n_sub * 4)), dim3(256), 0, st, strip, user,
                     p->d_sub_user.as<i64>(), p->d_sub_strip.as<i64>(), p->d_sub_shape.as<i32>(), p->n_sub);
}
template void strip_to_user<double>(const lsdm_pattern*, const double*, double*, hipStream_t);
template void strip_to_user<float>(const lsdm_pattern*, const float*, double*, hipStream_t);

template <class T>
void transpose_strips(const lsdm_pattern* p, const T* in, T* out, hipStream_t st) {
  ensure_maps(const_cast<lsdm_pattern*>(p));
  if (p->n_strips == 0) return;
  hipLaunchKernelGGL(k_transpose_strips<T>, dim3(grid_for(p->n_strips * 64)), dim3(256), 0, st, in, out,
                     p->d_mirror.as<i64>(), p->n_strips);
}
template void transpose_strips<double>(const lsdm_pattern*, const double*, double*, hipStream_t);
template void transpose_strips<float>(const lsdm_pattern*, const float*, float*, hipStream_t);

template <class T>
void sym_grad_to_user(const lsdm_pattern* p, const T* Lb, const T* V, double* user, hipStream_t st) {
  ensure_maps(const_cast<lsdm_pattern*>(p));
  if (p->n_sub == 0) return;
  hipLaunchKernelGGL(k_sym_grad_to_user<T>, dim3(grid_for(p->n_sub * 4)), dim3(256), 0, st, Lb, V, user,
                     p->d_sub_user.as<i64>(), p->d_sub_strip.as<i64>(), p->d_sub_shape.as<i32>(), p->n_sub,
                     p->d_mirror.as<i64>(), p->d_srow.as<i32>(), p->d_squad.as<i32>(), p->d_simg.as<i32>());
}
template void sym_grad_to_user<double>(const lsdm_pattern*, const double*, const double*, double*, hipStream_t);
template void sym_grad_to_user<float>(const lsdm_pattern*, const float*, const float*, double*, hipStream_t);

template <class T>
void sym_fill(const lsdm_pattern* p, T* data, hipStream_t st) {
  ensure_maps(const_cast<lsdm_pattern*>(p));
  if (p->n_fill == 0) return;
  hipLaunchKernelGGL(k_sym_fill<T>, dim3(grid_for(p->n_fill * 16)), dim3(256), 0, st, data, p->d_fill.as<i64>(),
                     p->d_mirror.as<i64>(), p->n_fill);
}
template void sym_fill<double>(const lsdm_pattern*, double*, hipStream_t);
template void sym_fill<float>(const lsdm_pattern*, float*, hipStream_t);
template void sym_fill<unsigned short>(const lsdm_pattern*, unsigned short*, hipStream_t);

void ensure_mirw(lsdm_pattern* p) {
  ensure_maps(p);
  std::lock_guard<std::mutex> lk(p->maps_mutex);
  if (p->mirw_ready) return;
  if (!mirw_fits(p))
    LSDM_THROW(LSDM_EUNSUPPORTED, "internal: pattern too large for mirror writes in the product epilogue");
  p->d_mirw.alloc(sizeof(i32) * std::max<i64>(1, 4 * p->n_strips));
  if (p->n_strips) {
    hipLaunchKernelGGL(k_mirw, dim3(grid_for(4 * p->n_strips)), dim3(256), 0, 0, p->d_srow.as<i32>(),
                       p->d_squad.as<i32>(), p->d_simg.as<i32>(), p->d_smask.as<uint8_t>(), p->d_mirror.as<i64>(),
                       p->d_mirw.as<i32>(), p->n_strips);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipDeviceSynchronize());
  }
  p->mirw_ready = true;
}

// Grid of the group kernel: as many workgroups as are resident at once (so
// every workgroup of an XCD walks its tile range in step with the others), a
// multiple of 8 (one contiguous tile range per XCD).
template <class K>
static unsigned gproduct_grid(K kernel, i64 ntiles) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;   // (kernel, device) -> resident workgroups
  int d = 0;
  HIP_CHECK(hipGetDevice(&d));
  int resident;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({reinterpret_cast<const void*>(kernel), d});
    if (it == cache.end()) {
      int per_cu = 0, cus = 0;
      HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0));
      HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d));
      it = cache.emplace(std::make_pair(reinterpret_cast<const void*>(kernel), d), std::max(1, per_cu) * std::max(1, cus)).first;
    }
    resident = it->second;
  }
  i64 blocks = std::min<i64>((ntiles + 7) / 8 * 8, resident);
  blocks = std::max<i64>(8, blocks / 8 * 8);
  return (unsigned)blocks;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

template <class T>
void product(const lsdm_plan* pl, const T* A, const T* B, T* C, double alpha, double beta, hipStream_t st,
             const T* Cin, const i64* cmap, bool mirrors) {
  const i32* mirw = nullptr;
  if (mirrors) {
    if (!pl->half || beta != 0.0 || cmap)
      LSDM_THROW(LSDM_EINVAL, "internal: mirror writes need a half-output plan without a beta term");
    ensure_mirw(const_cast<lsdm_pattern*>(pl->C));
    mirw = pl->C->d_mirw.as<i32>();
  }
  if (pl->n_gtiles == 0) return;
  const uint8_t* cm = pl->C->d_smask.as<uint8_t>();
  const GTile* Tl = pl->d_gtiles.as<GTile>();
  const GStep* S = pl->d_gsteps.as<GStep>();
  const dim3 b(256);
  // operand array bounds for the index clamp (a plan with steps has both)
  const int na = (int)std::max<i64>(1, pl->A->n_strips * 4), nbs = (int)std::max<i64>(1, pl->B->n_strips);
  unsigned long long* q = pl->d_queue.as<unsigned long long>();
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, q, 8);
  if (pl->transA)
    hipLaunchKernelGGL((k_gprod<T, true>), dim3(gproduct_grid(k_gprod<T, true>, pl->n_gtiles)), b, 0, st, Tl,
                       pl->n_gtiles, S, A, B, C, cm, (T)alpha, (T)beta, na, nbs, q, Cin, cmap, mirw);
  else
    hipLaunchKernelGGL((k_gprod<T, false>), dim3(gproduct_grid(k_gprod<T, false>, pl->n_gtiles)), b, 0, st, Tl,
                       pl->n_gtiles, S, A, B, C, cm, (T)alpha, (T)beta, na, nbs, q, Cin, cmap, mirw);
}
template void product<double>(const lsdm_plan*, const double*, const double*, double*, double, double, hipStream_t,
                              const double*, const i64*, bool);
template void product<float>(const lsdm_plan*, const float*, const float*, float*, double, double, hipStream_t,
                             const float*, const i64*, bool);


void plan_gsteps(const GTile* tiles, i64 ntiles, const GKEnt* kent, const i64* kbeg, const PlanView& v, int fill,
                 i32* counts, GStep* steps, unsigned long long* work) {
  if (ntiles == 0) return;
  i64 blocks = (ntiles + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_plan_gsteps, dim3((unsigned)blocks), dim3(256), 0, 0, tiles, ntiles, kent, kbeg, v, fill,
                     counts, steps, work);
}

static PatDev patdev(const lsdm_pattern* p) {
  return PatDev{p->d_sptr.as<i64>(), p->d_squad.as<i32>(), p->d_simg.as<i32>(), p->d_smask.as<uint8_t>()};
}

void offsite_f32(const lsdm_pattern* p, const double* in, float* out, hipStream_t st) {
  if (p->n_strips == 0) return;
  hipLaunchKernelGGL(k_offsite_f32, dim3(grid_for(p->n_strips * 64)), dim3(256), 0, st, in, out, p->d_srow.as<i32>(),
                     p->d_squad.as<i32>(), p->d_simg.as<i32>(), p->sys->d_patom.as<i32>(), p->n_strips);
}

static void rc_maps(lsdm_plan* pl) {
  std::lock_guard<std::mutex> lk(pl->rc_mutex);
  if (pl->rc_ready) return;
  const lsdm_pattern* C = pl->C;
  const lsdm_system* s = C->sys;
  int np = 1;
  for (i32 v : s->npseudo) np = std::max(np, (int)v);
  pl->rc_np = np;
  pl->d_rc_b.alloc(sizeof(i32) * std::max<i64>(1, C->n_strips * 4 * np));
  pl->d_rc_a.alloc(sizeof(i32) * std::max<i64>(1, C->n_strips * 4 * np));
  pl->d_rc_aon.alloc(sizeof(i32) * std::max<i64>(1, (i64)s->n_pseudo * np));
  pl->d_rc_bon.alloc(sizeof(i32) * std::max<i64>(1, (i64)s->n_pseudo * np));
  const dim3 b(256);
  if (C->n_strips) {
    if (pl->transA)
      hipLaunchKernelGGL((k_rc_map<true>), dim3(grid_for(C->n_strips * 4)), b, 0, 0, patdev(pl->A), patdev(pl->B),
                         patdev(C), C->d_srow.as<i32>(), s->d_patom.as<i32>(), s->d_pbase.as<i32>(),
                         s->d_npseudo.as<i32>(), np, C->n_strips, pl->d_rc_b.as<i32>(), pl->d_rc_a.as<i32>());
    else
      hipLaunchKernelGGL((k_rc_map<false>), dim3(grid_for(C->n_strips * 4)), b, 0, 0, patdev(pl->A), patdev(pl->B),
                         patdev(C), C->d_srow.as<i32>(), s->d_patom.as<i32>(), s->d_pbase.as<i32>(),
                         s->d_npseudo.as<i32>(), np, C->n_strips, pl->d_rc_b.as<i32>(), pl->d_rc_a.as<i32>());
  }
  if (pl->transA)
    hipLaunchKernelGGL((k_rc_onsite<true>), dim3(grid_for((i64)s->n_pseudo * np)), b, 0, 0, patdev(pl->A),
                       patdev(pl->B), s->d_patom.as<i32>(), s->d_pbase.as<i32>(), s->d_npseudo.as<i32>(), np,
                       s->n_pseudo, pl->d_rc_aon.as<i32>(), pl->d_rc_bon.as<i32>());
  else
    hipLaunchKernelGGL((k_rc_onsite<false>), dim3(grid_for((i64)s->n_pseudo * np)), b, 0, 0, patdev(pl->A),
                       patdev(pl->B), s->d_patom.as<i32>(), s->d_pbase.as<i32>(), s->d_npseudo.as<i32>(), np,
                       s->n_pseudo, pl->d_rc_aon.as<i32>(), pl->d_rc_bon.as<i32>());
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipDeviceSynchronize());
  pl->rc_ready = true;
}

void rc_correct(const lsdm_plan* cpl, const double* A64, const double* B64, const float* RR, double* C64, double alpha,
                double beta, hipStream_t st) {
  lsdm_plan* pl = const_cast<lsdm_plan*>(cpl);
  const lsdm_pattern* C = pl->C;
  if (C->n_strips == 0) return;
  rc_maps(pl);
  const lsdm_system* s = C->sys;
  const dim3 g(grid_for(C->n_strips * 64)), b(256);
  if (pl->transA)
    hipLaunchKernelGGL((k_rc_apply<true>), g, b, 0, st, C->d_smask.as<uint8_t>(), C->d_srow.as<i32>(),
                       C->d_squad.as<i32>(), C->d_simg.as<i32>(), s->d_patom.as<i32>(), pl->rc_np,
                       pl->d_rc_b.as<i32>(), pl->d_rc_a.as<i32>(), pl->d_rc_aon.as<i32>(), pl->d_rc_bon.as<i32>(), A64,
                       B64, RR, C64, C->n_strips, alpha, beta, pl->half);
  else
    hipLaunchKernelGGL((k_rc_apply<false>), g, b, 0, st, C->d_smask.as<uint8_t>(), C->d_srow.as<i32>(),
                       C->d_squad.as<i32>(), C->d_simg.as<i32>(), s->d_patom.as<i32>(), pl->rc_np,
                       pl->d_rc_b.as<i32>(), pl->d_rc_a.as<i32>(), pl->d_rc_aon.as<i32>(), pl->d_rc_bon.as<i32>(), A64,
                       B64, RR, C64, C->n_strips, alpha, beta, pl->half);
}

void to_bf16(const float* in, unsigned short* outR, unsigned short* outC, i64 n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n)), dim3(256), 0, st, in, outR, outC, n);
}

void user_to_bf16(const lsdm_pattern* p, const double* user, unsigned short* outR, unsigned short* outC,
                  hipStream_t st) {
  ensure_maps(const_cast<lsdm_pattern*>(p));
  if (p->n_sub == 0) return;
  hipLaunchKernelGGL(k_user_to_bf16, dim3(grid_for(p->n_sub * 4)), dim3(256), 0, st, user, outR, outC,
                     p->d_sub_user.as<i64>(), p->d_sub_strip.as<i64>(), p->d_sub_shape.as<i32>(), p->n_sub);
}

void product_bf16(const lsdm_plan* pl, const unsigned short* A, const unsigned short* B, float* C, double alpha,
                  double beta, hipStream_t st, unsigned short* outR, unsigned short* outC, const uint8_t* cneed,
                  const float* Cin, const i64* cmap) {
  if (pl->n_gtiles == 0) return;
  const GTile* Tl = pl->d_gtiles.as<GTile>();
  const GStep* S = pl->d_gsteps.as<GStep>();
  const uint8_t* cm = pl->C->d_smask.as<uint8_t>();
  const dim3 b(256);
  unsigned long long* q = pl->d_queue.as<unsigned long long>();
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, q, 8);
  // half plans write the mirrors of their block-transposed copy
  const i64* cmir = nullptr;
  if (pl->half && outC) {
    ensure_maps(const_cast<lsdm_pattern*>(pl->C));
    cmir = pl->C->d_mirror.as<i64>();
  }
  const i32* csq = pl->C->d_squad.as<i32>();
  const i32* csi = pl->C->d_simg.as<i32>();
  if (pl->transA)
    hipLaunchKernelGGL((k_gprod_bf16<true>), dim3(gproduct_grid(k_gprod_bf16<true>, pl->n_gtiles)), b, 0, st, Tl,
                       pl->n_gtiles, S, A, B, C, outR, outC, cm, (float)alpha, (float)beta, q, cmir, csq, csi, cneed, Cin, cmap);
  else
    hipLaunchKernelGGL((k_gprod_bf16<false>), dim3(gproduct_grid(k_gprod_bf16<false>, pl->n_gtiles)), b, 0, st, Tl,
                       pl->n_gtiles, S, A, B, C, outR, outC, cm, (float)alpha, (float)beta, q, cmir, csq, csi, cneed, Cin, cmap);
}

template <class T>
void kassembly_on(const lsdm_pattern* out, const i64* map, const T* M, const T* P, double* K, hipStream_t st,
                  const lsdm_pattern* Mpat) {
  const i64 n = out->n_strips;
  if (n == 0) return;
  KSym sym{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (Mpat) {
    ensure_maps(const_cast<lsdm_pattern*>(out));
    ensure_maps(const_cast<lsdm_pattern*>(Mpat));
    sym = KSym{Mpat->d_mirror.as<i64>(), out->d_mirror.as<i64>(), out->d_srow.as<i32>(), out->d_squad.as<i32>(),
               out->d_simg.as<i32>()};
  }
  hipLaunchKernelGGL(k_kassembly<T>, dim3(grid_for(n * 64)), dim3(256), 0, st, M, P, K, map,
                     out->d_smask.as<uint8_t>(), n, sym);
}
template void kassembly_on<double>(const lsdm_pattern*, const i64*, const double*, const double*, double*, hipStream_t,
                                   const lsdm_pattern*);
template void kassembly_on<float>(const lsdm_pattern*, const i64*, const float*, const float*, double*, hipStream_t,
                                  const lsdm_pattern*);

// in symmetric mode M and P may hold only their kept halves (see k_kassembly)
template <class T>
void kassembly(const lsdm_lnv* L, const T* M, const T* P, double* K, hipStream_t st) {
  kassembly_on<T>(L->pH, L->d_h2m.as<i64>(), M, P, K, st, L->sym ? L->pM : nullptr);
}
template void kassembly<double>(const lsdm_lnv*, const double*, const double*, double*, hipStream_t);
template void kassembly<float>(const lsdm_lnv*, const float*, const float*, double*, hipStream_t);

template <class T>
void scatter_h(const lsdm_lnv* L, const T* H, T* Mb, double scale, hipStream_t st) {
  const i64 nh = L->pH->n_strips;
  if (nh == 0) return;
  hipLaunchKernelGGL(k_scatter_h<T>, dim3(grid_for(nh * 64)), dim3(256), 0, st, H, Mb, L->d_h2m.as<i64>(),
                     L->pM->d_smask.as<uint8_t>(), nh, (T)scale);
}
template void scatter_h<double>(const lsdm_lnv*, const double*, double*, double, hipStream_t);
template void scatter_h<float>(const lsdm_lnv*, const float*, float*, double, hipStream_t);

template <class T>
void project_strips(const lsdm_pattern* out, const i64* map, const T* in, T* o, double scale, hipStream_t st) {
  const i64 n = out->n_strips;
  if (n == 0) return;
  hipLaunchKernelGGL(k_project_strips<T>, dim3(grid_for(n * 64)), dim3(256), 0, st, in, o, map,
                     out->d_smask.as<uint8_t>(), n, (T)scale);
}
template void project_strips<double>(const lsdm_pattern*, const i64*, const double*, double*, double, hipStream_t);
template void project_strips<float>(const lsdm_pattern*, const i64*, const float*, float*, double, hipStream_t);

// out = a x + b y (element-wise; out may be x or y)
__global__ void k_lincomb(double* out, const double* x, const double* y, double a, double b, i64 n) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < n; g += (i64)gridDim.x * blockDim.x)
    out[g] = a * x[g] + b * y[g];
}
void lincomb(double* out, const double* x, const double* y, double a, double b, i64 n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n)), dim3(256), 0, st, out, x, y, a, b, n);
}

// one wavefront per source block; the target blocks are distinct, so no two
// lanes write the same value
__global__ void k_add_blocks(double* out, const double* __restrict__ x, const i64* __restrict__ xoff,
                             const i64* __restrict__ hoff, const i32* __restrict__ size, i64 nb, double a) {
  const int lane = threadIdx.x & 63;
  const i64 nw = (i64)gridDim.x * (blockDim.x >> 6);
  for (i64 b = (blockIdx.x * (i64)blockDim.x + threadIdx.x) >> 6; b < nb; b += nw) {
    const i64 xo = xoff[b], ho = hoff[b];
    for (int e = lane; e < size[b]; e += 64) out[ho + e] += a * x[xo + e];
  }
}
void add_blocks(double* out, const double* x, const i64* xoff, const i64* hoff, const i32* size, i64 nb, double a,
                hipStream_t st) {
  if (nb <= 0) return;
  const i64 grid = std::min<i64>((nb + 3) / 4, 4096);
  hipLaunchKernelGGL(k_add_blocks, dim3((unsigned)grid), dim3(256), 0, st, out, x, xoff, hoff, size, nb, a);
}

// E from two compensated dots: s1 <a1, b1> + s2 <a2, b2>, the partial sums of
// each set merged in one pass (s1, s2 powers of two keep the merge exact)
__global__ void __launch_bounds__(256) k_dot_final2(const double* __restrict__ partial, int np, double s1,
                                                    double s2, double* __restrict__ out) {
  __shared__ double ss[256], sc[256];
  Comp acc{0.0, 0.0};
  for (int i = threadIdx.x; i < np; i += 256) {
    acc = comp_merge(acc, Comp{s1 * partial[2 * i], s1 * partial[2 * i + 1]});
    acc = comp_merge(acc, Comp{s2 * partial[2 * (np + i)], s2 * partial[2 * (np + i) + 1]});
  }
  ss[threadIdx.x] = acc.s;
  sc[threadIdx.x] = acc.c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      Comp m = comp_merge(Comp{ss[threadIdx.x], sc[threadIdx.x]}, Comp{ss[threadIdx.x + w], sc[threadIdx.x + w]});
      ss[threadIdx.x] = m.s;
      sc[threadIdx.x] = m.c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = ss[0] + sc[0];
}

void dot_parts(const double* a, const double* b, i64 n, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial<double>, dim3(DOT_BLOCKS), dim3(256), 0, st, a, b, n, partial);
}
void dot_final2(const double* partial, double s1, double s2, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_final2, dim3(1), dim3(256), 0, st, partial, DOT_BLOCKS, s1, s2, out);
}

void dot(const double* a, const double* b, i64 n, double scale, double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial<double>, dim3(DOT_BLOCKS), dim3(256), 0, st, a, b, n, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, partial, DOT_BLOCKS, scale, out);
}

// Scratch of the dot that allocates nothing (lsdm_dot_noalloc): the partial
// sums of the fixed grid, DOT_SCRATCH doubles (16 KiB), one copy per device,
// held until the process ends.  Every partial is written before it is read,
// so nothing needs clearing between calls; calls that overlap on one device
// share it and race.
static __device__ __align__(256) double scratch[DOT_SCRATCH];

double* dot_scratch() {
  static std::mutex mu;
  static std::map<int, double*> addr;   // device -> device address of `scratch`
  int d = 0;
  HIP_CHECK(hipGetDevice(&d));
  std::lock_guard<std::mutex> g(mu);
  auto it = addr.find(d);
  if (it != addr.end()) return it->second;
  // the array's name is a host-side stand-in; its address on device d comes
  // from the runtime, looked up once with d current
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    LSDM_THROW(LSDM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  addr.emplace(d, static_cast<double*>(ptr));
  return static_cast<double*>(ptr);
}

}  // namespace lsdm
