// Launchers of the HIP kernels (kernels.hip).
#pragma once
#include "lsdm_internal.h"

namespace lsdm {

constexpr int DOT_BLOCKS = 1024;   // fixed grid of the reproducible dot

template <class T> void fill(T* p, i64 n, T v, hipStream_t st);
template <class T> void user_to_strip(const lsdm_pattern* p, const double* user, T* strip, double scale, hipStream_t st);
template <class T> void strip_to_user(const lsdm_pattern* p, const T* strip, double* user, hipStream_t st);
template <class T> void transpose_strips(const lsdm_pattern* p, const T* in, T* out, hipStream_t st);
// C = alpha P_C(op(A) B) + beta C in strip layout (B already transposed if the plan says so)
template <class T> void product(const lsdm_plan* pl, const T* A, const T* B, T* C, double alpha, double beta, hipStream_t st);
template <class T> void kassembly(const lsdm_lnv* L, const T* M, const T* P, double* K, hipStream_t st);
template <class T> void scatter_h(const lsdm_lnv* L, const T* H, T* Mb, double scale, hipStream_t st);
// out[0] = scale * sum a[i] b[i]; partial holds 2 * DOT_BLOCKS doubles
void dot(const double* a, const double* b, i64 n, double scale, double* partial, double* out, hipStream_t st);

}  // namespace lsdm
