// HIP kernels of the lsdm library (gfx950).
//
//  * layout conversion between the caller's block layout and the internal
//    strip layout (gather/scatter of 4x4 sub-blocks);
//  * strip-layout transpose (B^T for products with a transposed B);
//  * the truncated block product C = alpha P_C(op(A) B) + beta C on MFMA:
//    one wavefront per tile of 4 output rows x 4 output column quads, 16
//    accumulator slots, one MFMA per active (row, column quad) slot per step;
//  * K assembly (eq. 3) and a bitwise-reproducible compensated FP64 dot.
//
// MFMA lane maps used below (measured on gfx950):
//   v_mfma_f64_4x4x4_4b_f64: lane l = 16k + 4b + x holds A[b][x][k] and
//     B[b][k][x]; the result D[b][r][c] is in lane 16r + 4b + c.
//   v_mfma_f32_4x4x1_16b_f32: lane l = 4b + x holds A[b][x][0] and B[b][0][x];
//     the result D[b][r][c] is in lane 4b + c, register r.
#include <hip/hip_runtime.h>

#include "kernels.h"

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

// one thread per element of every 4x4 sub-block of the map
template <class T>
__global__ void k_user_to_strip(const double* __restrict__ user, T* __restrict__ strip, const i64* __restrict__ su,
                                const i64* __restrict__ ss, const i32* __restrict__ sh, i64 nsub, double scale) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nsub * 16; g += (i64)gridDim.x * blockDim.x) {
    const i64 sb = g >> 4;
    const int e = (int)(g & 15), r = e >> 2, c = e & 3;
    const int shape = sh[sb], rows = shape & 255, cols = (shape >> 8) & 255, stride = shape >> 16;
    if (r < rows && c < cols) strip[ss[sb] + r * 4 + c] = (T)(scale * user[su[sb] + (i64)r * stride + c]);
  }
}

template <class T>
__global__ void k_strip_to_user(const T* __restrict__ strip, double* __restrict__ user, const i64* __restrict__ su,
                                const i64* __restrict__ ss, const i32* __restrict__ sh, i64 nsub) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nsub * 16; g += (i64)gridDim.x * blockDim.x) {
    const i64 sb = g >> 4;
    const int e = (int)(g & 15), r = e >> 2, c = e & 3;
    const int shape = sh[sb], rows = shape & 255, cols = (shape >> 8) & 255, stride = shape >> 16;
    if (r < rows && c < cols) user[su[sb] + (i64)r * stride + c] = (double)strip[ss[sb] + r * 4 + c];
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

// ---------------------------------------------------------------------------
// truncated block product, FP64: v_mfma_f64_4x4x4_4b_f64
// ---------------------------------------------------------------------------
template <bool TA>
__global__ void __launch_bounds__(256) k_prod_f64(const Tile* __restrict__ tiles, i64 ntiles,
                                                  const Step* __restrict__ steps, const double* __restrict__ A,
                                                  const double* __restrict__ B, double* __restrict__ C,
                                                  const uint8_t* __restrict__ cmask, double alpha, double beta) {
  const int lane = threadIdx.x & 63;
  const i64 wave0 = uniform64((i64)blockIdx.x * 4 + (threadIdx.x >> 6));
  const i64 nw = (i64)gridDim.x * 4;
  const int kk = lane >> 4, blk = (lane >> 2) & 3, x = lane & 3;
  // operand A[b][x][kk] = A_ik[x][kk]; transposed: (X_ki)^T[x][kk] = X_ki[kk][x]
  const int a_off = TA ? (kk * 4 + x) : (x * 4 + kk);
  // operand B[b][kk][x] = block b of the strip, element [kk][x]; the result
  // D[b][r][c] sits in lane 16r + 4b + c, which is the same offset
  const int b_off = blk * 16 + kk * 4 + x;
  for (i64 t = wave0; t < ntiles; t += nw) {
    const Tile* tp = tiles + t;
    const i64 s0 = tp->step0;
    const int ns = tp->nsteps;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    for (int s = 0; s < ns; ++s) {
      const Step* sp = steps + s0 + s;
      const uint32_t mask = sp->mask;
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const i32 a = sp->a[i];
        av[i] = a >= 0 ? A[(i64)a * 16 + a_off] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const i32 b = sp->b[j];
        bv[j] = b >= 0 ? B[(i64)b * 64 + b_off] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (mask >> (4 * i + j) & 1u) acc[4 * i + j] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[i], bv[j], acc[4 * i + j], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const i32 cs = tp->cstrip[q];
      if (cs < 0) continue;
      const bool keep = (cmask[cs] >> blk) & 1;
      const i64 idx = (i64)cs * 64 + b_off;
      double v = keep ? alpha * acc[q] : 0.0;
      if (beta != 0.0) v += beta * C[idx];
      C[idx] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// truncated block product, FP32: v_mfma_f32_4x4x1_16b_f32.  The 16 blocks of
// one instruction are (column block t, inner index kk) pairs b = 4t + kk; each
// holds the rank-1 term of one kk, and the 4 partials are summed across lanes
// at the end of the tile.  Lane l then loads and stores element l of a strip.
// ---------------------------------------------------------------------------
template <bool TA>
__global__ void __launch_bounds__(256) k_prod_f32(const Tile* __restrict__ tiles, i64 ntiles,
                                                  const Step* __restrict__ steps, const float* __restrict__ A,
                                                  const float* __restrict__ B, float* __restrict__ C,
                                                  const uint8_t* __restrict__ cmask, float alpha, float beta) {
  const int lane = threadIdx.x & 63;
  const i64 wave0 = uniform64((i64)blockIdx.x * 4 + (threadIdx.x >> 6));
  const i64 nw = (i64)gridDim.x * 4;
  const int x = lane & 3, kk = (lane >> 2) & 3, t4 = lane >> 4;
  const int a_off = TA ? (kk * 4 + x) : (x * 4 + kk);
  for (i64 t = wave0; t < ntiles; t += nw) {
    const Tile* tp = tiles + t;
    const i64 s0 = tp->step0;
    const int ns = tp->nsteps;
    f4 acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < ns; ++s) {
      const Step* sp = steps + s0 + s;
      const uint32_t mask = sp->mask;
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const i32 a = sp->a[i];
        av[i] = a >= 0 ? A[(i64)a * 16 + a_off] : 0.f;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const i32 b = sp->b[j];
        bv[j] = b >= 0 ? B[(i64)b * 64 + lane] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (mask >> (4 * i + j) & 1u) acc[4 * i + j] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[i], bv[j], acc[4 * i + j], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const i32 cs = tp->cstrip[q];
      if (cs < 0) continue;
      f4 v = acc[q];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] += __shfl_xor(v[e], 4);
        v[e] += __shfl_xor(v[e], 8);
      }
      const float r = kk == 0 ? v[0] : kk == 1 ? v[1] : kk == 2 ? v[2] : v[3];
      const bool keep = (cmask[cs] >> t4) & 1;
      const i64 idx = (i64)cs * 64 + lane;
      float o = keep ? alpha * r : 0.f;
      if (beta != 0.f) o += beta * C[idx];
      C[idx] = o;
    }
    (void)x;
  }
}

// ---------------------------------------------------------------------------
// K = 3 M|_H - 2 P on H's strips (FP64), masked to H's pattern
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_kassembly(const T* __restrict__ M, const T* __restrict__ P, double* __restrict__ K,
                            const i64* __restrict__ h2m, const uint8_t* __restrict__ hmask, i64 nh) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nh * 64; g += (i64)gridDim.x * blockDim.x) {
    const i64 h = g >> 6;
    const int e = (int)(g & 63), t = e >> 4;
    const bool in = (hmask[h] >> t) & 1;
    K[g] = in ? 3.0 * (double)M[h2m[h] * 64 + e] - 2.0 * (double)P[g] : 0.0;
  }
}

// Mbar = scale * H scattered into M's strips (the rest of Mbar is cleared first)
template <class T>
__global__ void k_scatter_h(const T* __restrict__ H, T* __restrict__ Mb, const i64* __restrict__ h2m, i64 nh, T scale) {
  for (i64 g = blockIdx.x * (i64)blockDim.x + threadIdx.x; g < nh * 64; g += (i64)gridDim.x * blockDim.x) {
    const i64 h = g >> 6;
    const int e = (int)(g & 63);
    Mb[h2m[h] * 64 + e] = scale * H[g];
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

template <class T>
void user_to_strip(const lsdm_pattern* p, const double* user, T* strip, double scale, hipStream_t st) {
  if (p->n_sub == 0) return;
  hipLaunchKernelGGL(k_user_to_strip<T>, dim3(grid_for(p->n_sub * 16)), dim3(256), 0, st, user, strip,
                     p->d_sub_user.as<i64>(), p->d_sub_strip.as<i64>(), p->d_sub_shape.as<i32>(), p->n_sub, scale);
}
template void user_to_strip<double>(const lsdm_pattern*, const double*, double*, double, hipStream_t);
template void user_to_strip<float>(const lsdm_pattern*, const double*, float*, double, hipStream_t);

template <class T>
void strip_to_user(const lsdm_pattern* p, const T* strip, double* user, hipStream_t st) {
  if (p->n_sub == 0) return;
  hipLaunchKernelGGL(k_strip_to_user<T>, dim3(grid_for(p->n_sub * 16)), dim3(256), 0, st, strip, user,
                     p->d_sub_user.as<i64>(), p->d_sub_strip.as<i64>(), p->d_sub_shape.as<i32>(), p->n_sub);
}
template void strip_to_user<double>(const lsdm_pattern*, const double*, double*, hipStream_t);
template void strip_to_user<float>(const lsdm_pattern*, const float*, double*, hipStream_t);

template <class T>
void transpose_strips(const lsdm_pattern* p, const T* in, T* out, hipStream_t st) {
  if (p->n_strips == 0) return;
  hipLaunchKernelGGL(k_transpose_strips<T>, dim3(grid_for(p->n_strips * 64)), dim3(256), 0, st, in, out,
                     p->d_mirror.as<i64>(), p->n_strips);
}
template void transpose_strips<double>(const lsdm_pattern*, const double*, double*, hipStream_t);
template void transpose_strips<float>(const lsdm_pattern*, const float*, float*, hipStream_t);

unsigned product_grid(i64 ntiles) {
  i64 blocks = (ntiles + 3) / 4;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

template <>
void product<double>(const lsdm_plan* pl, const double* A, const double* B, double* C, double alpha, double beta,
                     hipStream_t st) {
  if (pl->n_tiles == 0) return;
  const Tile* T = pl->d_tiles.as<Tile>();
  const Step* S = pl->d_steps.as<Step>();
  const uint8_t* cm = pl->C->d_smask.as<uint8_t>();
  if (pl->transA)
    hipLaunchKernelGGL(k_prod_f64<true>, dim3(product_grid(pl->n_tiles)), dim3(256), 0, st, T, pl->n_tiles, S, A, B, C, cm,
                       alpha, beta);
  else
    hipLaunchKernelGGL(k_prod_f64<false>, dim3(product_grid(pl->n_tiles)), dim3(256), 0, st, T, pl->n_tiles, S, A, B, C,
                       cm, alpha, beta);
}

template <>
void product<float>(const lsdm_plan* pl, const float* A, const float* B, float* C, double alpha, double beta,
                    hipStream_t st) {
  if (pl->n_tiles == 0) return;
  const Tile* T = pl->d_tiles.as<Tile>();
  const Step* S = pl->d_steps.as<Step>();
  const uint8_t* cm = pl->C->d_smask.as<uint8_t>();
  if (pl->transA)
    hipLaunchKernelGGL(k_prod_f32<true>, dim3(product_grid(pl->n_tiles)), dim3(256), 0, st, T, pl->n_tiles, S, A, B, C, cm,
                       (float)alpha, (float)beta);
  else
    hipLaunchKernelGGL(k_prod_f32<false>, dim3(product_grid(pl->n_tiles)), dim3(256), 0, st, T, pl->n_tiles, S, A, B, C,
                       cm, (float)alpha, (float)beta);
}

template <class T>
void kassembly(const lsdm_lnv* L, const T* M, const T* P, double* K, hipStream_t st) {
  const i64 nh = L->pH->n_strips;
  if (nh == 0) return;
  hipLaunchKernelGGL(k_kassembly<T>, dim3(grid_for(nh * 64)), dim3(256), 0, st, M, P, K, L->d_h2m.as<i64>(),
                     L->pH->d_smask.as<uint8_t>(), nh);
}
template void kassembly<double>(const lsdm_lnv*, const double*, const double*, double*, hipStream_t);
template void kassembly<float>(const lsdm_lnv*, const float*, const float*, double*, hipStream_t);

template <class T>
void scatter_h(const lsdm_lnv* L, const T* H, T* Mb, double scale, hipStream_t st) {
  const i64 nh = L->pH->n_strips;
  if (nh == 0) return;
  hipLaunchKernelGGL(k_scatter_h<T>, dim3(grid_for(nh * 64)), dim3(256), 0, st, H, Mb, L->d_h2m.as<i64>(), nh, (T)scale);
}
template void scatter_h<double>(const lsdm_lnv*, const double*, double*, double, hipStream_t);
template void scatter_h<float>(const lsdm_lnv*, const float*, float*, double, hipStream_t);

void dot(const double* a, const double* b, i64 n, double scale, double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial<double>, dim3(DOT_BLOCKS), dim3(256), 0, st, a, b, n, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, partial, DOT_BLOCKS, scale, out);
}

}  // namespace lsdm
