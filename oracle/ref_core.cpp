// Oracle core: plain FP64 CPU implementation of the atom-blocked truncated
// sparse products of the LNV density-matrix method.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link or call
// this file; only the tests, the smoke check and the CPU-baseline leg of the
// benchmark use it.  It shares no code with the GPU path.
//
// What it follows (Bowler & Miyazaki, "Calculations on millions of atoms with
// DFT: linear scaling shows its potential", section 2 "Methodology"):
//   * matrices are indexed by atom and support function (eq. 1, eq. 2), so a
//     matrix is a set of dense atom blocks nfn_i x nfn_j;
//   * locality: a block of a matrix of range R exists only for atom pairs at
//     distance <= R (the L cutoff stated just after eq. 3 makes an element zero
//     when the distance exceeds R_L; a pair at exactly R is kept);
//   * matrix multiplication is the main operation (item 1 of the list of
//     computational operations).  A truncated product is the exact product
//     projected on the output's range pattern: C = P_C(A B).
// Periodic systems are infinite crystals: a block is keyed by (i, j, n) with n
// an integer lattice translation applied to atom j, and
//   (A B)_{i,(j,n)} = sum over (k,m) of A_{i,(k,m)} B_{k,(j,n-m)}.
//
// Written for obviousness, not speed: one output row per loop iteration, a
// per-row lookup of the output slot, triple loops over block entries, and
// sequential compensated (Neumaier) sums for scalar reductions.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

typedef int64_t i64;
typedef int32_t i32;

namespace {

struct Pat {  // one range pattern in block-CSR form, rows sorted by (col, image)
  const i64* ptr; const i32* col; const i32* img; const i64* off; const uint8_t* present;
};

inline bool same_img(const i32* a, const i32 n0, const i32 n1, const i32 n2) {
  return a[0] == n0 && a[1] == n1 && a[2] == n2;
}

// index of block (j, n) in row i of pattern p, or -1
i64 find_block(const Pat& p, i64 i, i32 j, i32 n0, i32 n1, i32 n2) {
  i64 lo = p.ptr[i], hi = p.ptr[i + 1];
  while (lo < hi) {                       // lower bound on the column
    i64 mid = (lo + hi) / 2;
    if (p.col[mid] < j) lo = mid + 1; else hi = mid;
  }
  for (i64 b = lo; b < p.ptr[i + 1] && p.col[b] == j; ++b)
    if (same_img(p.img + 3 * b, n0, n1, n2)) return b;
  return -1;
}

void invert3(const double* T, double* inv) {
  double a = T[0], b = T[1], c = T[2], d = T[3], e = T[4], f = T[5], g = T[6], h = T[7], k = T[8];
  double det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
  inv[0] = (e * k - f * h) / det; inv[1] = (c * h - b * k) / det; inv[2] = (b * f - c * e) / det;
  inv[3] = (f * g - d * k) / det; inv[4] = (a * k - c * g) / det; inv[5] = (c * d - a * f) / det;
  inv[6] = (d * h - e * g) / det; inv[7] = (b * g - a * h) / det; inv[8] = (a * e - b * d) / det;
}

void note_missing(i64* missing, i64 row) {
#pragma omp critical(oracle_missing)
  if (*missing < 0 || row < *missing) *missing = row;
}

}  // namespace

extern "C" {

// Range pattern rows.  For every listed row atom i: all (j, n) with
// |x_j + n T - x_i|^2 <= R^2, in increasing (j, n0, n1, n2) order.
// lat: 9 doubles whose rows are the lattice vectors, or NULL (open system:
// only n = 0).  Count pass: row_ptr == NULL, fills counts[r].  Fill pass:
// writes col/img from row_ptr[r] on for row r.
int ref_pairs(i64 n_atoms, const double* xyz, const double* lat, double R, i64 nrows,
              const i64* rows, const i64* row_ptr, i64* counts, i32* col, i32* img) {
  double inv[9] = {0}, bnorm[3] = {0, 0, 0};
  if (lat) {
    invert3(lat, inv);
    // column k of inv is the reciprocal vector b_k; a vector v = (n + df) T has
    // coefficient (n + df)_k = v . b_k, so |n_k + df_k| <= |v| |b_k| <= R |b_k|
    for (int k = 0; k < 3; ++k)
      bnorm[k] = std::sqrt(inv[k] * inv[k] + inv[3 + k] * inv[3 + k] + inv[6 + k] * inv[6 + k]);
  }
  const double R2 = R * R;
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 r = 0; r < nrows; ++r) {
    const i64 i = rows[r];
    i64 w = row_ptr ? row_ptr[r] : 0, cnt = 0;
    const double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2];
    for (i64 j = 0; j < n_atoms; ++j) {
      const double dx0 = xyz[3 * j] - xi, dy0 = xyz[3 * j + 1] - yi, dz0 = xyz[3 * j + 2] - zi;
      int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      if (lat) {
        for (int k = 0; k < 3; ++k) {
          double df = dx0 * inv[k] + dy0 * inv[3 + k] + dz0 * inv[6 + k];
          lo[k] = (int)std::ceil(-df - R * bnorm[k]) - 1;   // one spare image each side;
          hi[k] = (int)std::floor(-df + R * bnorm[k]) + 1;  // the distance test decides
        }
      }
      for (int n0 = lo[0]; n0 <= hi[0]; ++n0)
        for (int n1 = lo[1]; n1 <= hi[1]; ++n1)
          for (int n2 = lo[2]; n2 <= hi[2]; ++n2) {
            double dx = dx0, dy = dy0, dz = dz0;
            if (lat) {
              dx = dx0 + ((double)n0 * lat[0] + (double)n1 * lat[3] + (double)n2 * lat[6]);
              dy = dy0 + ((double)n0 * lat[1] + (double)n1 * lat[4] + (double)n2 * lat[7]);
              dz = dz0 + ((double)n0 * lat[2] + (double)n1 * lat[5] + (double)n2 * lat[8]);
            }
            if (dx * dx + dy * dy + dz * dz <= R2) {
              if (row_ptr) {
                col[w] = (i32)j; img[3 * w] = n0; img[3 * w + 1] = n1; img[3 * w + 2] = n2; ++w;
              }
              ++cnt;
            }
          }
    }
    if (!row_ptr) counts[r] = cnt;
  }
  return 0;
}

// C = P_C(A B) on the present rows of C, accumulated into c_val (zero it first
// for a plain product).  Every A row needed (the present rows of C) and every B
// row reached (the columns k of those A rows) must be present; otherwise the
// call returns -(1 + lowest missing row) and the result is incomplete.
// If n_triples is not NULL it receives the number of block triples (i,k,j)
// that contributed.
int ref_multiply(i64 n_atoms, const i32* nfn,
                 const i64* a_ptr, const i32* a_col, const i32* a_img, const i64* a_off, const uint8_t* a_pres, const double* a_val,
                 const i64* b_ptr, const i32* b_col, const i32* b_img, const i64* b_off, const uint8_t* b_pres, const double* b_val,
                 const i64* c_ptr, const i32* c_col, const i32* c_img, const i64* c_off, const uint8_t* c_pres, double* c_val,
                 i64* n_triples) {
  const Pat A{a_ptr, a_col, a_img, a_off, a_pres}, B{b_ptr, b_col, b_img, b_off, b_pres}, C{c_ptr, c_col, c_img, c_off, c_pres};
  i64 missing = -1, triples = 0;
#pragma omp parallel reduction(+ : triples)
  {
    std::vector<i64> first(n_atoms, -1);   // first slot of column j in the current row of C
#pragma omp for schedule(dynamic, 4)
    for (i64 i = 0; i < n_atoms; ++i) {
      if (!C.present[i]) continue;
      if (!A.present[i]) { note_missing(&missing, i); continue; }
      for (i64 s = C.ptr[i + 1] - 1; s >= C.ptr[i]; --s) first[C.col[s]] = s;
      const int ni = nfn[i];
      for (i64 a = A.ptr[i]; a < A.ptr[i + 1]; ++a) {
        const i32 k = A.col[a];
        const i32 m0 = A.img[3 * a], m1 = A.img[3 * a + 1], m2 = A.img[3 * a + 2];
        if (!B.present[k]) { note_missing(&missing, k); continue; }
        const int nk = nfn[k];
        const double* Ab = a_val + A.off[a];
        for (i64 b = B.ptr[k]; b < B.ptr[k + 1]; ++b) {
          const i32 j = B.col[b];
          // image of atom j seen from row i: m + n'
          const i32 n0 = m0 + B.img[3 * b], n1 = m1 + B.img[3 * b + 1], n2 = m2 + B.img[3 * b + 2];
          i64 s = first[j];
          if (s < 0) continue;
          for (; s < C.ptr[i + 1] && C.col[s] == j; ++s)
            if (same_img(C.img + 3 * s, n0, n1, n2)) break;
          if (s >= C.ptr[i + 1] || C.col[s] != j) continue;   // outside C's range: truncated
          const int nj = nfn[j];
          const double* Bb = b_val + B.off[b];
          double* Cb = c_val + C.off[s];
          for (int r = 0; r < ni; ++r)
            for (int c = 0; c < nj; ++c) {
              double acc = 0.0;
              for (int q = 0; q < nk; ++q) acc += Ab[r * nk + q] * Bb[q * nj + c];
              Cb[r * nj + c] += acc;
            }
          ++triples;
        }
      }
      for (i64 s = C.ptr[i]; s < C.ptr[i + 1]; ++s) first[C.col[s]] = -1;
    }
  }
  if (n_triples) *n_triples = triples;
  return missing >= 0 ? (int)-(1 + missing) : 0;
}

// C = P_C(A B^T) on the present rows of C, accumulated into c_val:
//   C_{i,(j,n)} = sum over blocks (k,m) of A's row i of A_{i,(k,m)} (B_{j,(k,m-n)})^T
// since (B^T)_{(k,m),(j,n)} = (B_{(j,n),(k,m)})^T = (B_{j,(k,m-n)})^T.
// Rows i of A and rows j of B (the columns of C's present rows) must be
// present.  Row i of A and row j of B are both sorted by (k, image), and the
// shift m -> m - n keeps that order, so the pairs are found by a merge.
int ref_multiply_nt(i64 n_atoms, const i32* nfn,
                    const i64* a_ptr, const i32* a_col, const i32* a_img, const i64* a_off, const uint8_t* a_pres, const double* a_val,
                    const i64* b_ptr, const i32* b_col, const i32* b_img, const i64* b_off, const uint8_t* b_pres, const double* b_val,
                    const i64* c_ptr, const i32* c_col, const i32* c_img, const i64* c_off, const uint8_t* c_pres, double* c_val,
                    i64* n_triples) {
  const Pat A{a_ptr, a_col, a_img, a_off, a_pres}, B{b_ptr, b_col, b_img, b_off, b_pres}, C{c_ptr, c_col, c_img, c_off, c_pres};
  i64 missing = -1, triples = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : triples)
  for (i64 i = 0; i < n_atoms; ++i) {
    if (!C.present[i]) continue;
    if (!A.present[i]) { note_missing(&missing, i); continue; }
    const int ni = nfn[i];
    for (i64 s = C.ptr[i]; s < C.ptr[i + 1]; ++s) {
      const i32 j = C.col[s];
      if (!B.present[j]) { note_missing(&missing, j); continue; }
      const int nj = nfn[j];
      const i32 n0 = C.img[3 * s], n1 = C.img[3 * s + 1], n2 = C.img[3 * s + 2];
      double* Cb = c_val + C.off[s];
      i64 a = A.ptr[i], b = B.ptr[j];
      while (a < A.ptr[i + 1] && b < B.ptr[j + 1]) {
        // compare (k_a, m_a - n) with (k_b, m_b) lexicographically
        long ka[4] = {A.col[a], (long)A.img[3 * a] - n0, (long)A.img[3 * a + 1] - n1, (long)A.img[3 * a + 2] - n2};
        long kb[4] = {B.col[b], B.img[3 * b], B.img[3 * b + 1], B.img[3 * b + 2]};
        int cmp = 0;
        for (int t = 0; t < 4 && cmp == 0; ++t) cmp = (ka[t] < kb[t]) ? -1 : (ka[t] > kb[t]) ? 1 : 0;
        if (cmp < 0) { ++a; continue; }
        if (cmp > 0) { ++b; continue; }
        const int nk = nfn[A.col[a]];
        const double* Ab = a_val + A.off[a];
        const double* Bb = b_val + B.off[b];
        for (int r = 0; r < ni; ++r)
          for (int c = 0; c < nj; ++c) {
            double acc = 0.0;
            for (int q = 0; q < nk; ++q) acc += Ab[r * nk + q] * Bb[c * nk + q];
            Cb[r * nj + c] += acc;
          }
        ++triples; ++a; ++b;
      }
    }
  }
  if (n_triples) *n_triples = triples;
  return missing >= 0 ? (int)-(1 + missing) : 0;
}

// T = A^T on the present rows of T: block (i, j, n) of T is the transpose of
// block (j, i, -n) of A.  Rows j of A must be present.  A block of T whose
// mirror is absent from A's pattern is zero.
int ref_transpose(i64 n_atoms, const i32* nfn,
                  const i64* a_ptr, const i32* a_col, const i32* a_img, const i64* a_off, const uint8_t* a_pres, const double* a_val,
                  const i64* t_ptr, const i32* t_col, const i32* t_img, const i64* t_off, const uint8_t* t_pres, double* t_val) {
  const Pat A{a_ptr, a_col, a_img, a_off, a_pres}, T{t_ptr, t_col, t_img, t_off, t_pres};
  i64 missing = -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 i = 0; i < n_atoms; ++i) {
    if (!T.present[i]) continue;
    const int ni = nfn[i];
    for (i64 t = T.ptr[i]; t < T.ptr[i + 1]; ++t) {
      const i32 j = T.col[t];
      const int nj = nfn[j];
      double* Tb = t_val + T.off[t];
      if (!A.present[j]) { note_missing(&missing, j); continue; }
      i64 a = find_block(A, j, (i32)i, -T.img[3 * t], -T.img[3 * t + 1], -T.img[3 * t + 2]);
      for (int r = 0; r < ni; ++r)
        for (int c = 0; c < nj; ++c)
          Tb[r * nj + c] = (a < 0) ? 0.0 : a_val[A.off[a] + c * ni + r];
    }
  }
  return missing >= 0 ? (int)-(1 + missing) : 0;
}

// Q = P_Q(A): copy every block of A's pattern that lies in Q's pattern, zero
// elsewhere.  Rows of A must be present for the present rows of Q.
int ref_project(i64 n_atoms, const i32* nfn,
                const i64* a_ptr, const i32* a_col, const i32* a_img, const i64* a_off, const uint8_t* a_pres, const double* a_val,
                const i64* q_ptr, const i32* q_col, const i32* q_img, const i64* q_off, const uint8_t* q_pres, double* q_val) {
  const Pat A{a_ptr, a_col, a_img, a_off, a_pres}, Q{q_ptr, q_col, q_img, q_off, q_pres};
  i64 missing = -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 i = 0; i < n_atoms; ++i) {
    if (!Q.present[i]) continue;
    if (!A.present[i]) { note_missing(&missing, i); continue; }
    for (i64 q = Q.ptr[i]; q < Q.ptr[i + 1]; ++q) {
      const int sz = nfn[i] * nfn[Q.col[q]];
      i64 a = find_block(A, i, Q.col[q], Q.img[3 * q], Q.img[3 * q + 1], Q.img[3 * q + 2]);
      for (int e = 0; e < sz; ++e) q_val[Q.off[q] + e] = (a < 0) ? 0.0 : a_val[A.off[a] + e];
    }
  }
  return missing >= 0 ? (int)-(1 + missing) : 0;
}

// sum_k a[k] b[k] with Neumaier's compensated summation, sequential order.
double ref_dot(i64 n, const double* a, const double* b) {
  double s = 0.0, c = 0.0;
  for (i64 k = 0; k < n; ++k) {
    const double x = a[k] * b[k];
    const double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
  }
  return s + c;
}

}  // extern "C"
