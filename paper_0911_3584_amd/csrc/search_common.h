// Cell-list neighbour search of a range pattern (the locality cutoff stated
// after eq. 3: blocks (i, j, n) with |x_j + n T - x_i| <= R), shared by the
// host search and the GPU search so that both visit the same partners.
#pragma once
#include "lsdm_internal.h"

namespace lsdm {

// cells of width >= R (or R/k grids when the cell is large): nb cells per
// axis, D cells searched each way, the lattice T (rows) when periodic
struct SearchGeom {
  int nb[3];
  int D[3];
  int periodic;
  double lat[9];
  double R2;
};

// Every partner (j, image m0 m1 m2) of atom i within R, passed to visit.
// bin: cell coordinates of each atom; wrap: its lattice cell (periodic);
// cstart/catom: atoms of each cell (CSR).
template <class V>
__host__ __device__ inline void search_partners(const SearchGeom& g, i64 i, const double* xyz, const int* wrap,
                                                const int* bin, const i64* cstart, const i32* catom, V&& visit) {
  for (int d0 = -g.D[0]; d0 <= g.D[0]; ++d0)
    for (int d1 = -g.D[1]; d1 <= g.D[1]; ++d1)
      for (int d2 = -g.D[2]; d2 <= g.D[2]; ++d2) {
        int t[3] = {bin[3 * i] + d0, bin[3 * i + 1] + d1, bin[3 * i + 2] + d2}, sh[3] = {0, 0, 0};
        bool skip = false;
        for (int k = 0; k < 3; ++k) {
          if (g.periodic) {
            const int q = (t[k] >= 0) ? t[k] / g.nb[k] : -((-t[k] + g.nb[k] - 1) / g.nb[k]);
            sh[k] = q;
            t[k] -= q * g.nb[k];
          } else if (t[k] < 0 || t[k] >= g.nb[k]) {
            skip = true;
          }
        }
        if (skip) continue;
        const i64 c = ((i64)t[0] * g.nb[1] + t[1]) * g.nb[2] + t[2];
        for (i64 u = cstart[c]; u < cstart[c + 1]; ++u) {
          const i32 j = catom[u];
          int m0 = 0, m1 = 0, m2 = 0;
          if (g.periodic) {
            m0 = sh[0] - wrap[3 * j] + wrap[3 * i];
            m1 = sh[1] - wrap[3 * j + 1] + wrap[3 * i + 1];
            m2 = sh[2] - wrap[3 * j + 2] + wrap[3 * i + 2];
          }
          if (pair_dist2(xyz + 3 * i, xyz + 3 * j, m0, m1, m2, g.periodic ? g.lat : nullptr) <= g.R2)
            visit(j, m0, m1, m2);
        }
      }
}

}  // namespace lsdm

namespace lsdm {

// The search on the GPU (pattern.hip): per atom the partner count, then the
// partners as keys (j << 24 | packed image), each row sorted.  row_ptr
// (n + 1) and keys are host arrays filled here.  Throws LSDM_EUNSUPPORTED for
// an image index beyond +-127 and LSDM_ENOMEM when the pattern would reach
// 2^31 blocks (checked on the counts, before any row is stored).
void pattern_search_gpu(const SearchGeom& g, const double* xyz, const int* wrap, const int* bin, const i64* cstart,
                        const i32* catom, i32 n, i64 ncell, std::vector<i64>& row_ptr,
                        std::vector<unsigned long long>& keys);

}  // namespace lsdm
