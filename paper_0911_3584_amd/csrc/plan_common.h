// Step generation of a product plan, shared by the GPU kernel (kernels.hip)
// and the host path used when no device is present (symbolic.cpp).
//
// For a group tile (4*GQ output rows x GJ output column quads) and one entry
// of the group's inner list (pseudo-atom k with image m, and the A blocks of
// the rows), the B strip reaching column quad jq is (k, Q_jq, n_jq - m); slot
// (r, jq) is active when A_{r,k} exists and the strip holds a block (k, j)
// whose pair (r, j) is in C's pattern.
#pragma once
#include "lsdm_internal.h"

namespace lsdm {

// read-only views used by step generation
struct PlanView {
  const i64* b_sptr;
  const i32* b_squad;
  const i32* b_simg;
  const uint8_t* b_smask;
  const i32* c_squad;
  const i32* c_simg;
  const uint8_t* c_smask;
  const i32* prows;       // real rows of each pseudo-atom
  const uint8_t* first;   // 1 if the pseudo-atom is the first one of its atom
};

__host__ __device__ inline i32 img_sub(i32 a, i32 b) { return img_add(a, img_neg(b)); }

// B strip of row k with key `key`, or -1
__host__ __device__ inline i64 find_b_strip(const PlanView& v, i32 k, i64 key) {
  i64 lo = v.b_sptr[k], hi = v.b_sptr[k + 1];
  while (lo < hi) {
    const i64 mid = (lo + hi) >> 1;
    const i64 kk = skey(v.b_squad[mid], v.b_simg[mid]);
    if (kk < key) lo = mid + 1; else hi = mid;
  }
  if (lo < v.b_sptr[k + 1] && skey(v.b_squad[lo], v.b_simg[lo]) == key) return lo;
  return -1;
}

// ---------------------------------------------------------------------------
// group tiles: GQ row quads share one inner list
// ---------------------------------------------------------------------------
struct GKEnt {
  i32 k;
  i32 m;
  i32 a[GROWS];
};

__host__ __device__ inline i64 gtile_column_key(const PlanView& v, const GTile& t, int jq) {
  for (int r = 0; r < GROWS; ++r) {
    const i32 cs = t.cstrip[GJ * r + jq];
    if (cs >= 0) return skey(v.c_squad[cs], v.c_simg[cs]);
  }
  return -1;
}

// Work of one (group tile, inner entry, column quad): B strip index, slot bits
// per wavefront (bit GJ*i + jq of mask[w] for row 4w+i), useful flops and
// atom triples.
__host__ __device__ inline void gslot_work(const PlanView& v, const GTile& t, const GKEnt& e, int jq, i64 colkey,
                                           i32* bidx, uint32_t (&mask)[GQ], uint64_t* flops, uint64_t* triples) {
  *bidx = -1;
  for (int w = 0; w < GQ; ++w) mask[w] = 0;
  if (colkey < 0) return;
  const i32 q = (i32)(colkey >> 24), n = (i32)(colkey & 0xffffff);
  const i64 b = find_b_strip(v, e.k, skey(q, img_sub(n, e.m)));
  if (b < 0) return;
  *bidx = (i32)b;
  const uint8_t bm = v.b_smask[b];
  for (int r = 0; r < GROWS; ++r) {
    if (e.a[r] < 0) continue;
    const i32 cs = t.cstrip[GJ * r + jq];
    if (cs < 0) continue;
    const uint8_t u = bm & v.c_smask[cs];
    if (!u) continue;
    mask[r >> 2] |= 1u << (GJ * (r & 3) + jq);
    const i32 pi = GROWS * t.group + r;
    for (int bb = 0; bb < 4; ++bb) {
      if (!(u >> bb & 1)) continue;
      const i32 pj = 4 * q + bb;
      *flops += 2ull * (uint64_t)v.prows[pi] * (uint64_t)v.prows[e.k] * (uint64_t)v.prows[pj];
      if (v.first[pi] && v.first[e.k] && v.first[pj]) *triples += 1;
    }
  }
}

}  // namespace lsdm
