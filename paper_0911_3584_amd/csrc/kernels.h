// Launchers of the HIP kernels (kernels.hip).
#pragma once
#include "lsdm_internal.h"
#include "plan_common.h"

namespace lsdm {

constexpr int DOT_BLOCKS = 1024;   // fixed grid of the reproducible dot
constexpr int DOT_SCRATCH = 2 * DOT_BLOCKS;   // partial sums of one dot (doubles)
// device address, on the current device, of the dot's static scratch (looked
// up on the first call per device)
double* dot_scratch();

// layout maps of a pattern (built on first use; symbolic.cpp)
void ensure_maps(lsdm_pattern* p);
void ensure_mirw(lsdm_pattern* p);
// the mirror words (block index + 1 in 31 bits) reach every block of the pattern
inline bool mirw_fits(const lsdm_pattern* p) { return 4 * p->n_strips < ((i64)1 << 30); }

template <class T> void fill(T* p, i64 n, T v, hipStream_t st);
template <class T> void user_to_strip(const lsdm_pattern* p, const double* user, T* strip, double scale, hipStream_t st);
template <class T> void strip_to_user(const lsdm_pattern* p, const T* strip, double* user, hipStream_t st);
template <class T> void transpose_strips(const lsdm_pattern* p, const T* in, T* out, hipStream_t st);
// the strips of a symmetric result outside keep_strip, as transposes of their mirrors
template <class T> void sym_fill(const lsdm_pattern* p, T* data, hipStream_t st);
// out += v + v^T (strip layout, every block of p)
// dE/dL of symmetric mode into the caller's layout: Lbar (kept half) + V + V^T
template <class T> void sym_grad_to_user(const lsdm_pattern* p, const T* Lb, const T* V, double* user, hipStream_t st);
// C = alpha P_C(op(A) B) + beta C in strip layout (B already transposed if the plan says so);
// with cmap (C strip -> Cin strip, nullable) the beta term is beta Cin on the mapped strips,
// masked to C's blocks, instead of beta C.  mirrors (half-output plan, beta = 0): the epilogue
// also writes the dropped half, every present block's transpose into its mirror (what
// sym_fill would copy); absent blocks of dropped strips are not written
template <class T>
void product(const lsdm_plan* pl, const T* A, const T* B, T* C, double alpha, double beta, hipStream_t st,
             const T* Cin = nullptr, const i64* cmap = nullptr, bool mirrors = false);
// symbolic pass on the GPU: steps of a plan (count pass fill = 0, fill pass fill = 1)
void plan_gsteps(const GTile* tiles, i64 ntiles, const GKEnt* kent, const i64* kbeg, const PlanView& v, int fill,
                 i32* counts, GStep* steps, unsigned long long* work);
// zero records after the last group step (the product kernel stages records
// up to two batches past a tile's end)
constexpr i64 GSTEP_PAD = 32;
// residual mode: fp32 copy of the off-site part; FP64 correction
// C = alpha (RR + D_A B + A D_B - D_A D_B) + beta C with RR = P_C(R_A R_B) in fp32
void offsite_f32(const lsdm_pattern* p, const double* in, float* out, hipStream_t st);
void rc_correct(const lsdm_plan* pl, const double* A64, const double* B64, const float* RR, double* C64, double alpha,
                double beta, hipStream_t st);
// BF16 path: fp32 strips -> bf16 copies (row-major R and/or block-transposed C)
void to_bf16(const float* in, unsigned short* outR, unsigned short* outC, i64 n, hipStream_t st);
// caller's block layout (FP64) -> bf16 strip copies (R and/or C, either null)
void user_to_bf16(const lsdm_pattern* p, const double* user, unsigned short* outR, unsigned short* outC,
                  hipStream_t st);
// C (fp32) = alpha P_C(op(A) B) + beta C with bf16 operands (A: R copy, or C copy of X when transposed; B: C copy);
// C may be null when only the bf16 copies of the result are wanted (outR, outC: nullable, written from the
// FP32 result in the product's epilogue); cneed (nullable, a byte per C strip) limits the FP32 writes to the
// strips marked.  A half plan's outC also receives the copy's dropped half (mirrors of the kept blocks).
void product_bf16(const lsdm_plan* pl, const unsigned short* A, const unsigned short* B, float* C, double alpha,
                  double beta, hipStream_t st, unsigned short* outR = nullptr, unsigned short* outC = nullptr,
                  const uint8_t* cneed = nullptr, const float* Cin = nullptr, const i64* cmap = nullptr);
template <class T> void kassembly(const lsdm_lnv* L, const T* M, const T* P, double* K, hipStream_t st);
// K = 3 M|_out - 2 P on an output pattern: map[s] = M's strip with out's strip s key
template <class T>
void kassembly_on(const lsdm_pattern* out, const i64* map, const T* M, const T* P, double* K, hipStream_t st,
                  const lsdm_pattern* Mpat = nullptr);
template <class T> void scatter_h(const lsdm_lnv* L, const T* H, T* Mb, double scale, hipStream_t st);
// o = scale * P_out(in) in strip layout: out's strip s from in's strip map[s], masked to out's blocks
template <class T>
void project_strips(const lsdm_pattern* out, const i64* map, const T* in, T* o, double scale, hipStream_t st);
// out[0] = scale * sum a[i] b[i]; partial holds 2 * DOT_BLOCKS doubles
void dot(const double* a, const double* b, i64 n, double scale, double* partial, double* out, hipStream_t st);
// partial sums of <a, b> (DOT_BLOCKS pairs), and s1 <first set> + s2 <second set> at partial + 2 DOT_BLOCKS
void dot_parts(const double* a, const double* b, i64 n, double* partial, hipStream_t st);
void dot_final2(const double* partial, double s1, double s2, double* out, hipStream_t st);
// out = a x + b y, n doubles
void lincomb(double* out, const double* x, const double* y, double a, double b, i64 n, hipStream_t st);
// out[hoff[b] + e] += a * x[xoff[b] + e] for e < size[b], b < nb (distinct target blocks)
void add_blocks(double* out, const double* x, const i64* xoff, const i64* hoff, const i32* size, i64 nb, double a,
                hipStream_t st);

}  // namespace lsdm
