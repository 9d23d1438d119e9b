// GPU neighbour search of range patterns (symbolic pass, step 1): the cell
// list is built on the host; every atom's partners are counted, then written
// as (j, image) keys and sorted per row with rocPRIM's segmented radix sort
// (hipCUB interface).  The walk and the range test are those of the host
// search (search_common.h).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "search_common.h"

namespace lsdm {

constexpr i64 PATTERN_MAX_BLOCKS = (i64)1 << 31;

// one thread per atom; FILL = 0 counts (and flags images beyond +-127, which
// both passes skip), FILL = 1 writes the keys of row i from row_ptr[i]
template <int FILL>
__global__ void __launch_bounds__(64) k_pattern_search(SearchGeom g, const double* __restrict__ xyz,
                                                       const int* __restrict__ wrap, const int* __restrict__ bin,
                                                       const i64* __restrict__ cstart, const i32* __restrict__ catom,
                                                       i32 n, i64* __restrict__ cnt, const i64* __restrict__ row_ptr,
                                                       unsigned long long* __restrict__ keys, int* __restrict__ bad) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
    i64 c = 0;
    i64 w = FILL ? row_ptr[i] : 0;
    search_partners(g, i, xyz, wrap, bin, cstart, catom, [&](i32 j, int m0, int m1, int m2) {
      if (m0 < -127 || m0 > 127 || m1 < -127 || m1 > 127 || m2 < -127 || m2 > 127) {
        if (!FILL) atomicOr(bad, 1);
        return;
      }
      if (FILL)
        keys[w++] = ((unsigned long long)(unsigned)j << 24) | (unsigned long long)(unsigned)img_pack(m0, m1, m2);
      else
        ++c;
    });
    if (!FILL) cnt[i] = c;
  }
}

void pattern_search_gpu(const SearchGeom& g, const double* xyz, const int* wrap, const int* bin, const i64* cstart,
                        const i32* catom, i32 n, i64 ncell, std::vector<i64>& row_ptr,
                        std::vector<unsigned long long>& keys) {
  DevBuf d_xyz, d_wrap, d_bin, d_cstart, d_catom, d_cnt, d_bad, d_rp;
  d_xyz.upload(xyz, sizeof(double) * 3 * (size_t)n);
  d_wrap.upload(wrap, sizeof(int) * 3 * (size_t)n);
  d_bin.upload(bin, sizeof(int) * 3 * (size_t)n);
  d_cstart.upload(cstart, sizeof(i64) * (size_t)(ncell + 1));
  d_catom.upload(catom, sizeof(i32) * (size_t)n);
  d_cnt.alloc(sizeof(i64) * (size_t)n);
  const int zero = 0;
  d_bad.upload(&zero, sizeof(int));
  const unsigned grid = (unsigned)std::max<i64>(1, std::min<i64>((n + 63) / 64, 65536));
  hipLaunchKernelGGL(k_pattern_search<0>, dim3(grid), dim3(64), 0, 0, g, d_xyz.as<double>(), d_wrap.as<int>(),
                     d_bin.as<int>(), d_cstart.as<i64>(), d_catom.as<i32>(), n, d_cnt.as<i64>(), nullptr, nullptr,
                     d_bad.as<int>());
  HIP_CHECK(hipGetLastError());
  std::vector<i64> cnt((size_t)n);
  int bad = 0;
  HIP_CHECK(hipMemcpy(cnt.data(), d_cnt.p, sizeof(i64) * (size_t)n, hipMemcpyDeviceToHost));
  HIP_CHECK(hipMemcpy(&bad, d_bad.p, sizeof(int), hipMemcpyDeviceToHost));
  if (bad) LSDM_THROW(LSDM_EUNSUPPORTED, "lattice image index beyond +-127");
  row_ptr.assign((size_t)n + 1, 0);
  for (i32 a = 0; a < n; ++a) row_ptr[a + 1] = row_ptr[a] + cnt[a];
  const i64 total = row_ptr[n];
  if (total >= PATTERN_MAX_BLOCKS) LSDM_THROW(LSDM_ENOMEM, "pattern exceeds 2^31 blocks (range too large for the system)");
  keys.assign((size_t)total, 0ull);
  if (total == 0) return;
  d_rp.upload(row_ptr.data(), sizeof(i64) * row_ptr.size());
  DevBuf d_k, d_k2, d_tmp;
  d_k.alloc(sizeof(unsigned long long) * (size_t)total);
  d_k2.alloc(sizeof(unsigned long long) * (size_t)total);
  hipLaunchKernelGGL(k_pattern_search<1>, dim3(grid), dim3(64), 0, 0, g, d_xyz.as<double>(), d_wrap.as<int>(),
                     d_bin.as<int>(), d_cstart.as<i64>(), d_catom.as<i32>(), n, nullptr, d_rp.as<i64>(),
                     d_k.as<unsigned long long>(), nullptr);
  HIP_CHECK(hipGetLastError());
  // keys hold j (< n) above 24 bits of image: sort only the bits in use
  int end_bit = 24;
  while (end_bit < 64 && ((unsigned long long)(n - 1) >> (end_bit - 24)) != 0) ++end_bit;
  size_t tmp_bytes = 0;
  HIP_CHECK(hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, tmp_bytes, d_k.as<unsigned long long>(),
                                                       d_k2.as<unsigned long long>(), (int)total, n,
                                                       d_rp.as<i64>(), d_rp.as<i64>() + 1, 0, end_bit));
  d_tmp.alloc(std::max<size_t>(tmp_bytes, 16));
  HIP_CHECK(hipcub::DeviceSegmentedRadixSort::SortKeys(d_tmp.p, tmp_bytes, d_k.as<unsigned long long>(),
                                                       d_k2.as<unsigned long long>(), (int)total, n,
                                                       d_rp.as<i64>(), d_rp.as<i64>() + 1, 0, end_bit));
  HIP_CHECK(hipMemcpy(keys.data(), d_k2.p, sizeof(unsigned long long) * (size_t)total, hipMemcpyDeviceToHost));
}

}  // namespace lsdm
