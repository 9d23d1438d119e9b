// Symbolic pass, host side: system ordering, range patterns (cell-list
// neighbour search), the strip layout of a pattern and the tile/step task
// lists of truncated products.
//
// Source of the operations: Bowler & Miyazaki, section 2.  A range pattern is
// the set of atom pairs within the cutoff (stated after eq. 3); a truncated
// product keeps only the output blocks of its own range pattern.  Atoms are
// ordered along a Hilbert curve, as the paper's partitioner orders atoms into
// partitions (Results, strong scaling); here the order serves the MFMA
// kernels: consecutive pseudo-atoms are close in space, so the 4x4 block
// groups (quads) and the 16-atom row groups of a tile are compact and share
// neighbours.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <mutex>
#include <unordered_map>

#include "kernels.h"
#include "lsdm_internal.h"
#include "plan_common.h"
#include "search_common.h"

namespace lsdm {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
template <class F>
void parallel_for(i64 n, F&& f, int grain = 16) {
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (n < 2 * grain || nt == 1) {
    for (i64 i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<i64> next(0);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (;;) {
        i64 s = next.fetch_add(grain);
        if (s >= n) break;
        i64 e = std::min(n, s + (i64)grain);
        for (i64 i = s; i < e; ++i) f(i);
      }
    });
  for (auto& t : th) t.join();
}

static void invert3(const double* T, double* inv) {
  double a = T[0], b = T[1], c = T[2], d = T[3], e = T[4], f = T[5], g = T[6], h = T[7], k = T[8];
  double det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
  if (!(std::fabs(det) > 0) || !std::isfinite(det)) LSDM_THROW(LSDM_EINVAL, "lattice is singular");
  inv[0] = (e * k - f * h) / det; inv[1] = (c * h - b * k) / det; inv[2] = (b * f - c * e) / det;
  inv[3] = (f * g - d * k) / det; inv[4] = (a * k - c * g) / det; inv[5] = (c * d - a * f) / det;
  inv[6] = (d * h - e * g) / det; inv[7] = (b * g - a * h) / det; inv[8] = (a * e - b * d) / det;
}

static uint64_t spread3(uint64_t v) {  // 21 bits -> every third bit
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

// Position of the point (x0, x1, x2) (each `bits` bits) along a 3-D Hilbert
// curve, by Skilling's transform of the coordinates into the transposed
// Hilbert index (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc.
// 707, 2004), whose bits are then interleaved, x0's first.
static uint64_t hilbert3(uint64_t x0, uint64_t x1, uint64_t x2, int bits) {
  uint64_t X[3] = {x0, x1, x2};
  const uint64_t M = (uint64_t)1 << (bits - 1);
  for (uint64_t Q = M; Q > 1; Q >>= 1) {           // undo the excess work of the inverse
    const uint64_t P = Q - 1;
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const uint64_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];                                     // Gray encode
  X[2] ^= X[1];
  uint64_t t = 0;
  for (uint64_t Q = M; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  for (int i = 0; i < 3; ++i) X[i] ^= t;
  return (spread3(X[0]) << 2) | (spread3(X[1]) << 1) | spread3(X[2]);
}

// ---------------------------------------------------------------------------
// system: Hilbert order and pseudo-atoms
// ---------------------------------------------------------------------------
void build_system(lsdm_system* s) {
  const i32 n = s->n_atoms;
  std::vector<double> f(3 * (size_t)n);
  if (s->periodic) {
    invert3(s->lat, s->inv);
    for (i32 a = 0; a < n; ++a)
      for (int k = 0; k < 3; ++k) {
        double v = s->xyz[3 * a] * s->inv[k] + s->xyz[3 * a + 1] * s->inv[3 + k] + s->xyz[3 * a + 2] * s->inv[6 + k];
        f[3 * a + k] = v - std::floor(v);
      }
  } else {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (i32 a = 0; a < n; ++a)
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], s->xyz[3 * a + k]);
        hi[k] = std::max(hi[k], s->xyz[3 * a + k]);
      }
    double span = 1e-30;
    for (int k = 0; k < 3; ++k) span = std::max(span, hi[k] - lo[k]);
    for (i32 a = 0; a < n; ++a)
      for (int k = 0; k < 3; ++k) f[3 * a + k] = (s->xyz[3 * a + k] - lo[k]) / span;
  }
  std::vector<uint64_t> code(n);
  const double scale = (double)((1 << 21) - 1);
  for (i32 a = 0; a < n; ++a) {
    uint64_t q[3];
    for (int k = 0; k < 3; ++k) q[k] = (uint64_t)std::min(scale, std::max(0.0, std::floor(f[3 * a + k] * scale)));
    code[a] = hilbert3(q[0], q[1], q[2], 21);
  }
  s->order.resize(n);
  std::iota(s->order.begin(), s->order.end(), 0);
  std::stable_sort(s->order.begin(), s->order.end(), [&](i32 x, i32 y) { return code[x] < code[y]; });
  s->pbase.assign(n, 0);
  s->npseudo.assign(n, 0);
  s->patom.clear();
  s->prows.clear();
  for (i32 pos = 0; pos < n; ++pos) {
    i32 a = s->order[pos];
    i32 np = (s->nfn[a] + 3) / 4;
    s->pbase[a] = (i32)s->patom.size();
    s->npseudo[a] = np;
    for (i32 t = 0; t < np; ++t) {
      s->patom.push_back(a);
      s->prows.push_back(std::min(4, s->nfn[a] - 4 * t));
    }
  }
  while (s->patom.size() % 4) {  // padding pseudo-atoms: no rows, no blocks
    s->patom.push_back(-1);
    s->prows.push_back(0);
  }
  s->n_pseudo = (i32)s->patom.size();
  s->n_quads = s->n_pseudo / 4;
  s->first.assign(s->n_pseudo, 0);
  for (i32 q = 0; q < s->n_pseudo; ++q) s->first[q] = (s->patom[q] >= 0 && s->pbase[s->patom[q]] == q) ? 1 : 0;
  s->d_prows.upload(s->prows.data(), sizeof(i32) * s->prows.size());
  s->d_first.upload(s->first.data(), s->first.size());
  s->d_patom.upload(s->patom.data(), sizeof(i32) * s->patom.size());
  s->d_pbase.upload(s->pbase.data(), sizeof(i32) * s->pbase.size());
  s->d_npseudo.upload(s->npseudo.data(), sizeof(i32) * s->npseudo.size());
}

// ---------------------------------------------------------------------------
// range pattern, block layout: cell-list neighbour search
//   all (i, j, n) with |x_j + n T - x_i|^2 <= R^2, rows sorted by (j, n)
// Atoms are binned on fractional coordinates with bins wider than R across
// each pair of lattice planes, so every partner lies within D bins (D = 1
// unless the cell is thinner than R, when the bin/image pairs wrap around).
// The distance is evaluated from the caller's positions as
//   (x_j - x_i) + (n0 T0 + n1 T1 + n2 T2), component by component.
// ---------------------------------------------------------------------------
bool have_device();

void build_pattern_blocks(lsdm_pattern* p) {
  const lsdm_system* s = p->sys;
  const i32 n = s->n_atoms;
  const double R = p->R, R2 = R * R;
  int nb[3] = {1, 1, 1}, D[3] = {1, 1, 1};
  std::vector<int> wrap(3 * (size_t)n, 0);
  std::vector<int> bin(3 * (size_t)n, 0);
  if (s->periodic) {
    for (int k = 0; k < 3; ++k) {
      const double bn = std::sqrt(s->inv[k] * s->inv[k] + s->inv[3 + k] * s->inv[3 + k] + s->inv[6 + k] * s->inv[6 + k]);
      const double w = 1.0 / bn;   // distance between the lattice planes of axis k
      const double width = std::max(R * (1.0 + 1e-9), 1e-300);
      nb[k] = (int)std::max(1.0, std::min(1024.0, std::floor(w / width)));
      const double Dk = std::floor(R * nb[k] / w) + 1.0;   // checked before the conversion to int
      if (!(2.0 * Dk + 1.0 <= 255.0)) LSDM_THROW(LSDM_EUNSUPPORTED, "range too large for the image encoding");
      D[k] = (int)Dk;
    }
    for (i32 a = 0; a < n; ++a)
      for (int k = 0; k < 3; ++k) {
        double f = s->xyz[3 * a] * s->inv[k] + s->xyz[3 * a + 1] * s->inv[3 + k] + s->xyz[3 * a + 2] * s->inv[6 + k];
        double fl = std::floor(f);
        wrap[3 * a + k] = (int)fl;
        int b = (int)std::floor((f - fl) * nb[k]);
        bin[3 * a + k] = std::min(nb[k] - 1, std::max(0, b));
      }
  } else {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (i32 a = 0; a < n; ++a)
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], s->xyz[3 * a + k]);
        hi[k] = std::max(hi[k], s->xyz[3 * a + k]);
      }
    const double width = std::max(R * (1.0 + 1e-9), 1e-9);
    for (int k = 0; k < 3; ++k) nb[k] = (int)std::max(1.0, std::min(1024.0, std::floor((hi[k] - lo[k]) / width) + 1));
    for (i32 a = 0; a < n; ++a)
      for (int k = 0; k < 3; ++k)
        bin[3 * a + k] = std::min(nb[k] - 1, std::max(0, (int)std::floor((s->xyz[3 * a + k] - lo[k]) / width)));
  }
  const i64 ncell = (i64)nb[0] * nb[1] * nb[2];
  std::vector<i64> cstart(ncell + 1, 0);
  std::vector<i32> catom(n);
  auto cid = [&](int b0, int b1, int b2) { return ((i64)b0 * nb[1] + b1) * nb[2] + b2; };
  for (i32 a = 0; a < n; ++a) ++cstart[cid(bin[3 * a], bin[3 * a + 1], bin[3 * a + 2]) + 1];
  for (i64 c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
  {
    std::vector<i64> w(cstart.begin(), cstart.end() - 1);
    for (i32 a = 0; a < n; ++a) catom[w[cid(bin[3 * a], bin[3 * a + 1], bin[3 * a + 2])]++] = a;
  }
  SearchGeom geom;
  for (int k = 0; k < 3; ++k) {
    geom.nb[k] = nb[k];
    geom.D[k] = D[k];
  }
  geom.periodic = s->periodic ? 1 : 0;
  for (int k = 0; k < 9; ++k) geom.lat[k] = s->lat[k];
  geom.R2 = R2;
  if (have_device()) {
    // the GPU search: counts, the block-index limit, then the sorted rows
    std::vector<unsigned long long> keys;
    pattern_search_gpu(geom, s->xyz.data(), wrap.data(), bin.data(), cstart.data(), catom.data(), n, ncell,
                       p->row_ptr, keys);
    const i64 nbk = p->row_ptr[n];
    p->col.resize(nbk);
    p->img.resize(nbk);
    parallel_for(n, [&](i64 a) {
      for (i64 w = p->row_ptr[a]; w < p->row_ptr[a + 1]; ++w) {
        p->col[w] = (i32)(keys[w] >> 24);
        p->img[w] = (i32)(keys[w] & 0xffffff);
      }
    });
    return;
  }
  // every partner (j, image) of row i within R, passed to visit(j, m0, m1, m2)
  auto search_row = [&](i64 i, auto&& visit) {
    search_partners(geom, i, s->xyz.data(), wrap.data(), bin.data(), cstart.data(), catom.data(), visit);
  };
  // Size check before any row is stored: when the pair count could reach the
  // block-index limit (2^31 blocks; their values alone would then fill an
  // MI355X), count first, stopping as soon as the limit is passed.  The
  // estimate is the pair count of a uniform density over the cell (periodic)
  // or the bounding box (open), with a safety factor of 4.
  constexpr i64 MAX_BLOCKS = (i64)1 << 31;
  {
    double vol;
    if (s->periodic) {
      const double* T = s->lat;
      vol = std::fabs(T[0] * (T[4] * T[8] - T[5] * T[7]) - T[1] * (T[3] * T[8] - T[5] * T[6]) +
                      T[2] * (T[3] * T[7] - T[4] * T[6]));
    } else {
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (i32 a = 0; a < n; ++a)
        for (int k = 0; k < 3; ++k) {
          lo[k] = std::min(lo[k], s->xyz[3 * a + k]);
          hi[k] = std::max(hi[k], s->xyz[3 * a + k]);
        }
      vol = 1.0;
      for (int k = 0; k < 3; ++k) vol *= std::max(hi[k] - lo[k], 1.0);
    }
    const double ball = 4.18879020478639 * R * R * R;   // 4/3 pi R^3
    const double est = (double)n * (1.0 + (s->periodic ? (double)n * ball / vol : std::min((double)n, (double)n * ball / vol)));
    if (4.0 * est >= (double)MAX_BLOCKS) {
      std::atomic<i64> total(0);
      std::atomic<bool> over(false);
      parallel_for(n, [&](i64 i) {
        if (over.load(std::memory_order_relaxed)) return;
        i64 c = 0;
        search_row(i, [&](i32, int, int, int) { ++c; });
        if (total.fetch_add(c) + c >= MAX_BLOCKS) over = true;
      }, 8);
      if (over) LSDM_THROW(LSDM_ENOMEM, "pattern exceeds 2^31 blocks (range too large for the system)");
    }
  }
  std::vector<std::vector<std::pair<i64, i32>>> rows(n);   // ((j << 24) | img) per row
  std::atomic<int> bad(0);
  parallel_for(n, [&](i64 i) {
    auto& r = rows[i];
    search_row(i, [&](i32 j, int m0, int m1, int m2) {
      if (m0 < -127 || m0 > 127 || m1 < -127 || m1 > 127 || m2 < -127 || m2 > 127) {
        bad = 1;
        return;
      }
      r.push_back({((i64)j << 24) | img_pack(m0, m1, m2), 0});
    });
    std::sort(r.begin(), r.end());
  }, 8);
  if (bad) LSDM_THROW(LSDM_EUNSUPPORTED, "lattice image index beyond +-127");
  p->row_ptr.assign(n + 1, 0);
  for (i32 a = 0; a < n; ++a) p->row_ptr[a + 1] = p->row_ptr[a] + (i64)rows[a].size();
  const i64 nb_tot = p->row_ptr[n];
  if (nb_tot >= MAX_BLOCKS) LSDM_THROW(LSDM_ENOMEM, "pattern exceeds 2^31 blocks");
  p->col.resize(nb_tot);
  p->img.resize(nb_tot);
  parallel_for(n, [&](i64 a) {
    i64 w = p->row_ptr[a];
    for (auto& e : rows[a]) {
      p->col[w] = (i32)(e.first >> 24);
      p->img[w] = (i32)(e.first & 0xffffff);
      ++w;
    }
  });
}

// ---------------------------------------------------------------------------
// Structural pattern of a product: the blocks (i, k, n) of the sphere of
// p->R reachable as (A B)_{i,(k,n)} = sum over (l, m) of A_{i,(l,m)}
// B_{l,(k,n-m)}, or the same with A and B exchanged.  A product of matrices
// on these patterns is exactly zero on the other blocks of the sphere (no
// term reaches them), so they need no storage and no work; taking both orders
// keeps the pattern symmetric when A's and B's are (then the second set is the
// transpose of the first), which transposed uses of the product need.
// ---------------------------------------------------------------------------
void build_pattern_reach(lsdm_pattern* p, const lsdm_pattern* A, const lsdm_pattern* B) {
  build_pattern_blocks(p);   // the sphere
  const i32 n = p->sys->n_atoms;
  std::vector<std::vector<std::pair<i32, i32>>> rows(n);   // (col, img) kept per row
  parallel_for(n, [&](i64 i) {
    std::vector<i64> reach;
    for (int pass = 0; pass < 2; ++pass) {
      const lsdm_pattern* X = pass ? B : A;
      const lsdm_pattern* Y = pass ? A : B;
      for (i64 b = X->row_ptr[i]; b < X->row_ptr[i + 1]; ++b) {
        const i32 l = X->col[b], m = X->img[b];
        for (i64 c = Y->row_ptr[l]; c < Y->row_ptr[l + 1]; ++c)
          reach.push_back(((i64)Y->col[c] << 24) | img_add(m, Y->img[c]));
      }
    }
    std::sort(reach.begin(), reach.end());
    reach.erase(std::unique(reach.begin(), reach.end()), reach.end());
    auto& r = rows[i];
    for (i64 b = p->row_ptr[i]; b < p->row_ptr[i + 1]; ++b)
      if (std::binary_search(reach.begin(), reach.end(), ((i64)p->col[b] << 24) | p->img[b]))
        r.push_back({p->col[b], p->img[b]});
  }, 8);
  std::vector<i64> rp(n + 1, 0);
  for (i32 a = 0; a < n; ++a) rp[a + 1] = rp[a] + (i64)rows[a].size();
  p->row_ptr = rp;
  p->col.assign(rp[n], 0);
  p->img.assign(rp[n], 0);
  parallel_for(n, [&](i64 a) {
    i64 w = rp[a];
    for (auto& e : rows[a]) {
      p->col[w] = e.first;
      p->img[w] = e.second;
      ++w;
    }
  });
}

// ---------------------------------------------------------------------------
// strip layout of a pattern whose block layout (row_ptr, col, img) is filled
// ---------------------------------------------------------------------------
static i64 find_strip(const lsdm_pattern* p, i32 row, i64 key) {
  i64 lo = p->sptr[row], hi = p->sptr[row + 1];
  while (lo < hi) {
    i64 mid = (lo + hi) >> 1;
    i64 k = skey(p->squad[mid], p->simg[mid]);
    if (k < key) lo = mid + 1; else hi = mid;
  }
  if (lo < p->sptr[row + 1] && skey(p->squad[lo], p->simg[lo]) == key) return lo;
  return -1;
}

void build_strips(lsdm_pattern* p) {
  const lsdm_system* s = p->sys;
  const i32 n = s->n_atoms, np = s->n_pseudo;
  // block layout value offsets
  p->val_off.resize(p->col.size());
  i64 off = 0;
  for (i32 a = 0; a < n; ++a)
    for (i64 b = p->row_ptr[a]; b < p->row_ptr[a + 1]; ++b) {
      p->val_off[b] = off;
      off += (i64)s->nfn[a] * s->nfn[p->col[b]];
    }
  p->nval = off;
  // strips per pseudo-row: (quad, image) -> mask
  std::vector<std::vector<std::pair<i64, uint8_t>>> rows(np);
  parallel_for(n, [&](i64 a) {
    for (i32 sa = 0; sa < s->npseudo[a]; ++sa) {
      i32 pa = s->pbase[a] + sa;
      auto& r = rows[pa];
      for (i64 b = p->row_ptr[a]; b < p->row_ptr[a + 1]; ++b) {
        i32 j = p->col[b];
        for (i32 sb = 0; sb < s->npseudo[j]; ++sb) {
          i32 pb = s->pbase[j] + sb;
          r.push_back({skey(pb >> 2, p->img[b]), (uint8_t)(1u << (pb & 3))});
        }
      }
      std::sort(r.begin(), r.end());
      size_t w = 0;
      for (size_t t = 0; t < r.size(); ++t) {
        if (w > 0 && r[w - 1].first == r[t].first) r[w - 1].second |= r[t].second;
        else r[w++] = r[t];
      }
      r.resize(w);
    }
  });
  p->sptr.assign(np + 1, 0);
  for (i32 q = 0; q < np; ++q) p->sptr[q + 1] = p->sptr[q] + (i64)rows[q].size();
  p->n_strips = p->sptr[np];
  if (p->n_strips >= (i64)1 << 29) LSDM_THROW(LSDM_ENOMEM, "pattern too large for 32-bit strip indices");
  p->squad.resize(p->n_strips);
  p->simg.resize(p->n_strips);
  p->smask.resize(p->n_strips);
  parallel_for(np, [&](i64 q) {
    i64 w = p->sptr[q];
    for (auto& e : rows[q]) {
      p->squad[w] = (i32)(e.first >> 24);
      p->simg[w] = (i32)(e.first & 0xffffff);
      p->smask[w] = e.second;
      ++w;
    }
  });
  rows.clear();
  rows.shrink_to_fit();
  {
    std::vector<i32> srow(p->n_strips);
    for (i32 q = 0; q < np; ++q)
      for (i64 st = p->sptr[q]; st < p->sptr[q + 1]; ++st) srow[st] = q;
    p->d_srow.upload(srow.data(), sizeof(i32) * srow.size());
  }
  p->d_sptr.upload(p->sptr.data(), sizeof(i64) * p->sptr.size());
  p->d_squad.upload(p->squad.data(), sizeof(i32) * p->squad.size());
  p->d_simg.upload(p->simg.data(), sizeof(i32) * p->simg.size());
  p->d_smask.upload(p->smask.data(), p->smask.size());
}

// Maps needed only by patterns that cross the boundary or are transposed:
// block layout <-> strip layout (per 4x4 sub-block), on-site sub-blocks and
// the mirror map.  Built on first use.
void ensure_maps(lsdm_pattern* p) {
  std::lock_guard<std::mutex> lk(p->maps_mutex);
  if (p->maps_ready) return;
  const lsdm_system* s = p->sys;
  const i32 n = s->n_atoms, np = s->n_pseudo;
  // sub-block maps between the two layouts
  std::vector<i64> subcnt(n + 1, 0);
  for (i32 a = 0; a < n; ++a) {
    i64 c = 0;
    for (i64 b = p->row_ptr[a]; b < p->row_ptr[a + 1]; ++b) c += (i64)s->npseudo[a] * s->npseudo[p->col[b]];
    subcnt[a + 1] = subcnt[a] + c;
  }
  p->n_sub = subcnt[n];
  std::vector<i64> su(p->n_sub), ss(p->n_sub);
  std::vector<i32> sh(p->n_sub);
  parallel_for(n, [&](i64 a) {
    i64 w = subcnt[a];
    for (i64 b = p->row_ptr[a]; b < p->row_ptr[a + 1]; ++b) {
      i32 j = p->col[b];
      for (i32 sa = 0; sa < s->npseudo[a]; ++sa)
        for (i32 sb = 0; sb < s->npseudo[j]; ++sb) {
          i32 pa = s->pbase[a] + sa, pb = s->pbase[j] + sb;
          i64 st = find_strip(p, pa, skey(pb >> 2, p->img[b]));
          if (st < 0) LSDM_THROW(LSDM_EDEVICE, "internal: strip of a pattern block not found");
          su[w] = p->val_off[b] + (i64)(4 * sa) * s->nfn[j] + 4 * sb;
          ss[w] = st * 64 + (pb & 3) * 16;
          sh[w] = s->prows[pa] | (s->prows[pb] << 8) | (s->nfn[j] << 16);
          ++w;
        }
    }
  });
  p->d_sub_user.upload(su.data(), sizeof(i64) * su.size());
  p->d_sub_strip.upload(ss.data(), sizeof(i64) * ss.size());
  p->d_sub_shape.upload(sh.data(), sizeof(i32) * sh.size());
  // mirror map: block t of strip s in row q is (q, 4Q+t, n); its mirror is
  // (4Q+t, q, -n), found in strip (4Q+t, quad(q), -n) at block q & 3
  std::vector<i64> mir(4 * (size_t)p->n_strips, -1);
  parallel_for(np, [&](i64 q) {
    for (i64 st = p->sptr[q]; st < p->sptr[q + 1]; ++st)
      for (int t = 0; t < 4; ++t) {
        if (!(p->smask[st] >> t & 1)) continue;
        i32 r = 4 * p->squad[st] + t;
        const i64 ms = find_strip(p, r, skey((i32)(q >> 2), img_neg(p->simg[st])));
        mir[4 * st + t] = ms < 0 ? -1 : ms * 64 + (q & 3) * 16;
      }
  });
  p->d_mirror.upload(mir.data(), sizeof(i64) * mir.size());
  std::vector<i64> fl;
  for (i32 q = 0; q < np; ++q)
    for (i64 st = p->sptr[q]; st < p->sptr[q + 1]; ++st) {
      int m = 0;
      if (!keep_strip(q, p->squad[st], p->simg[st])) {
        m = 15;                       // every block: absent ones are written as zero
      } else if (p->squad[st] == (q >> 2) && p->simg[st] == IMG0) {
        for (int t = 0; t < 4; ++t)
          if (4 * p->squad[st] + t < q) m |= 1 << t;
        m &= p->smask[st];
      }
      if (m) fl.push_back((st << 4) | m);
    }
  p->n_fill = (i64)fl.size();
  p->d_fill.upload(fl.data(), sizeof(i64) * fl.size());
  p->maps_ready = true;
}

// ---------------------------------------------------------------------------
// product plan: tiles (4 output rows x up to TJ output column quads) and steps
//
// Host: per row quad, the inner list (union over its 4 rows of A's blocks
// (k, m), with each row's block) and the tiles (its output column quads in
// groups of TJ).  Device: the steps of every tile (k_plan_steps), so the task
// list, which is the bulk of a plan, never passes through host memory.
// ---------------------------------------------------------------------------

// Inner list of output rows row0 .. row0+NR-1: the union over the rows of A's
// blocks (k, m), one entry per (k, m) with the A block of every row (-1 where
// absent), sorted by (k, m).  For a transposed A the row pattern is A's own
// (range patterns are symmetric) and the block is the transpose of A_{k,(i,-m)}.
template <int NR, class Ent>
static void inner_list(const lsdm_pattern* A, bool tA, i32 row0, std::vector<Ent>& K) {
  const i32 np = A->sys->n_pseudo;
  std::vector<std::pair<i64, std::pair<int, i32>>> raw;
  for (int ii = 0; ii < NR; ++ii) {
    const i32 row = row0 + ii;
    if (row >= np) break;
    for (i64 st = A->sptr[row]; st < A->sptr[row + 1]; ++st)
      for (int t = 0; t < 4; ++t) {
        if (!(A->smask[st] >> t & 1)) continue;
        const i32 k = 4 * A->squad[st] + t;
        const i32 m = A->simg[st];
        i64 blk;
        if (!tA) {
          blk = st * 4 + t;
        } else {
          const i64 ms = find_strip(A, k, skey(row >> 2, img_neg(m)));
          if (ms < 0) LSDM_THROW(LSDM_EPATTERN, "transposed operand pattern is not symmetric");
          blk = ms * 4 + (row & 3);
        }
        raw.push_back({((i64)k << 24) | m, {ii, (i32)blk}});
      }
  }
  std::sort(raw.begin(), raw.end());
  K.clear();
  for (auto& e : raw) {
    if (K.empty() || (((i64)K.back().k << 24) | K.back().m) != e.first) {
      Ent ke;
      ke.k = (i32)(e.first >> 24);
      ke.m = (i32)(e.first & 0xffffff);
      for (int ii = 0; ii < NR; ++ii) ke.a[ii] = -1;
      K.push_back(ke);
    }
    K.back().a[e.second.first] = e.second.second;
  }
}

// sorted, distinct column keys of C's strips in rows row0 .. row0+nr-1 (only
// the kept half when `half`)
static std::vector<i64> column_keys(const lsdm_pattern* C, i32 row0, int nr, bool half) {
  std::vector<i64> ck;
  for (int ii = 0; ii < nr; ++ii) {
    const i32 row = row0 + ii;
    if (row >= C->sys->n_pseudo) break;
    for (i64 st = C->sptr[row]; st < C->sptr[row + 1]; ++st)
      if (!half || keep_strip(row, C->squad[st], C->simg[st])) ck.push_back(skey(C->squad[st], C->simg[st]));
  }
  std::sort(ck.begin(), ck.end());
  ck.erase(std::unique(ck.begin(), ck.end()), ck.end());
  return ck;
}

// Plan of a truncated product: group tiles of GQ row quads x GJ column quads
// (inner list: the union over the group's rows), steps generated on the GPU in
// two passes (count, then fill); without a device the host counts only.
void build_plan(lsdm_plan* pl) {
  const lsdm_pattern* A = pl->A;
  const lsdm_pattern* B = pl->B;
  const lsdm_pattern* C = pl->C;
  const lsdm_system* s = C->sys;
  const i32 ng = (s->n_quads + GQ - 1) / GQ;
  const bool tA = pl->transA != 0;
  std::vector<std::vector<GKEnt>> kents(ng);
  std::vector<std::vector<GTile>> tiles(ng);
  parallel_for(ng, [&](i64 g) {
    const i32 row0 = GROWS * (i32)g;
    inner_list<GROWS>(A, tA, row0, kents[g]);
    const bool half = pl->half != 0;
    const std::vector<i64> ckeys = column_keys(C, row0, GROWS, half);
    const i64 nt = ((i64)ckeys.size() + GJ - 1) / GJ;
    std::vector<GTile> T(nt);
    for (i64 t = 0; t < nt; ++t) {
      T[t].group = (i32)g;
      T[t].nsteps = 0;
      T[t].step0 = 0;
      for (int q = 0; q < GROWS * GJ; ++q) T[t].cstrip[q] = -1;
    }
    for (int r = 0; r < GROWS; ++r) {
      const i32 row = row0 + r;
      if (row >= s->n_pseudo) break;
      for (i64 st = C->sptr[row]; st < C->sptr[row + 1]; ++st) {
        if (half && !keep_strip(row, C->squad[st], C->simg[st])) continue;
        const i64 c = std::lower_bound(ckeys.begin(), ckeys.end(), skey(C->squad[st], C->simg[st])) - ckeys.begin();
        T[c / GJ].cstrip[GJ * r + (c % GJ)] = (i32)st;
      }
    }
    tiles[g] = std::move(T);
  }, 1);
  std::vector<i64> kbeg(ng + 1, 0);
  for (i32 g = 0; g < ng; ++g) kbeg[g + 1] = kbeg[g] + (i64)kents[g].size();
  std::vector<GKEnt> allK(kbeg[ng]);
  parallel_for(ng, [&](i64 g) { std::copy(kents[g].begin(), kents[g].end(), allK.begin() + kbeg[g]); });
  std::vector<std::vector<GKEnt>>().swap(kents);
  std::vector<GTile> allT;
  for (i32 g = 0; g < ng; ++g) allT.insert(allT.end(), tiles[g].begin(), tiles[g].end());
  std::vector<std::vector<GTile>>().swap(tiles);
  // Traversal order: super-groups of GSUPER groups, inside a super-group by
  // the tile's first output column, so the tiles that run together on one XCD
  // cover neighbouring rows and the same columns: they share B strips (same
  // columns) and A blocks (same rows) through its L2.
  {
    std::vector<std::pair<std::pair<i64, i64>, i64>> key(allT.size());
    for (size_t t = 0; t < allT.size(); ++t) {
      i64 c0 = -1;
      for (int q = 0; q < GROWS * GJ && c0 < 0; ++q)
        if (allT[t].cstrip[q] >= 0) c0 = skey(C->squad[allT[t].cstrip[q]], C->simg[allT[t].cstrip[q]]);
      key[t] = {{allT[t].group / GSUPER, c0}, (i64)t};
    }
    std::sort(key.begin(), key.end());
    std::vector<GTile> ord(allT.size());
    for (size_t t = 0; t < allT.size(); ++t) ord[t] = allT[key[t].second];
    allT.swap(ord);
  }
  const i64 ntile = (i64)allT.size();
  pl->n_gtiles = ntile;
  pl->d_queue.alloc(8 * sizeof(unsigned long long));
  if (have_device()) {
    DevBuf d_k, d_kb, d_cnt, d_work;
    d_k.upload(allK.data(), sizeof(GKEnt) * allK.size());
    d_kb.upload(kbeg.data(), sizeof(i64) * kbeg.size());
    pl->d_gtiles.upload(allT.data(), sizeof(GTile) * allT.size());
    d_cnt.alloc(sizeof(i32) * (ntile + 1));
    d_work.alloc(16);
    HIP_CHECK(hipMemset(d_work.p, 0, 16));
    PlanView v{B->d_sptr.as<i64>(), B->d_squad.as<i32>(), B->d_simg.as<i32>(), B->d_smask.as<uint8_t>(),
               C->d_squad.as<i32>(), C->d_simg.as<i32>(), C->d_smask.as<uint8_t>(), s->d_prows.as<i32>(),
               s->d_first.as<uint8_t>()};
    plan_gsteps(pl->d_gtiles.as<GTile>(), ntile, d_k.as<GKEnt>(), d_kb.as<i64>(), v, 0, d_cnt.as<i32>(), nullptr,
                d_work.as<unsigned long long>());
    HIP_CHECK(hipGetLastError());
    std::vector<i32> cnt(ntile);
    uint64_t work[2];
    if (ntile) HIP_CHECK(hipMemcpy(cnt.data(), d_cnt.p, sizeof(i32) * ntile, hipMemcpyDeviceToHost));
    HIP_CHECK(hipMemcpy(work, d_work.p, 16, hipMemcpyDeviceToHost));
    i64 nstep = 0;
    for (i64 t = 0; t < ntile; ++t) {
      allT[t].step0 = nstep;
      allT[t].nsteps = cnt[t];
      nstep += cnt[t];
    }
    pl->n_gsteps = nstep;
    pl->flops = (double)work[0];
    pl->n_triples = (i64)work[1];
    pl->d_gtiles.upload(allT.data(), sizeof(GTile) * allT.size());
    // the product kernel stages records up to two batches past a tile's last
    // step: pad with zero records
    pl->d_gsteps.alloc(sizeof(GStep) * (nstep + GSTEP_PAD));
    HIP_CHECK(hipMemset(pl->d_gsteps.p, 0, sizeof(GStep) * (nstep + GSTEP_PAD)));
    plan_gsteps(pl->d_gtiles.as<GTile>(), ntile, d_k.as<GKEnt>(), d_kb.as<i64>(), v, 1, nullptr,
                pl->d_gsteps.as<GStep>(), nullptr);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipDeviceSynchronize());
  } else {
    PlanView v{B->sptr.data(), B->squad.data(), B->simg.data(), B->smask.data(), C->squad.data(), C->simg.data(),
               C->smask.data(), s->prows.data(), s->first.data()};
    std::vector<i64> ns(ntile, 0);
    std::vector<uint64_t> fl(ntile, 0), tr(ntile, 0);
    parallel_for(ntile, [&](i64 t) {
      const GTile& tl = allT[t];
      i64 ck[GJ];
      for (int jq = 0; jq < GJ; ++jq) ck[jq] = gtile_column_key(v, tl, jq);
      for (i64 e = kbeg[tl.group]; e < kbeg[tl.group + 1]; ++e) {
        uint32_t any = 0;
        for (int jq = 0; jq < GJ; ++jq) {
          i32 b;
          uint32_t m[GQ];
          gslot_work(v, tl, allK[e], jq, ck[jq], &b, m, &fl[t], &tr[t]);
          for (int w = 0; w < GQ; ++w) any |= m[w];
        }
        if (any) ++ns[t];
      }
    }, 16);
    i64 nstep = 0;
    uint64_t F = 0, Tr = 0;
    for (i64 t = 0; t < ntile; ++t) {
      nstep += ns[t];
      F += fl[t];
      Tr += tr[t];
    }
    pl->n_gsteps = nstep;
    pl->flops = (double)F;
    pl->n_triples = (i64)Tr;
  }
}

}  // namespace lsdm
