// Internal data structures of the lsdm library (not part of the ABI).
//
// Internal layout ("strip layout").  Every atom is split into pseudo-atoms of
// at most 4 support functions (an atom with nfn = 13 becomes 4 pseudo-atoms,
// the last padded with 3 zero rows/columns), so all internal blocks are 4x4
// and match the 4x4x4 multi-block MFMA forms of gfx950.  Atoms are ordered
// along a Hilbert curve so that consecutive pseudo-atoms are spatially close;
// a "quad" is 4 consecutive pseudo-atoms.  A matrix row (one pseudo-atom) is
// stored as a list of strips, one per column quad (and lattice image) that
// holds at least one in-range pair: 4 blocks of 4x4 = 64 values, block t for
// pseudo-atom 4Q+t, zero where the pair is outside the range.  A 4-bit mask per
// strip records which of its blocks lie in the pattern.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lsdm.h"

namespace lsdm {

typedef int64_t i64;
typedef int32_t i32;

// -------- errors -----------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};
void set_error(int code, const std::string& msg);
#define LSDM_THROW(code, msg) throw ::lsdm::Error{(code), (msg)}
#define HIP_CHECK(x)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      LSDM_THROW(e_ == hipErrorOutOfMemory ? LSDM_ENOMEM : LSDM_EDEVICE,                 \
                 std::string(#x) + ": " + hipGetErrorString(e_));                        \
  } while (0)

// -------- device buffers ---------------------------------------------------
// Memory comes from hipMalloc or from the caller's allocator set with
// lsdm_set_allocator; a buffer keeps the release function of the allocator
// that made it.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  lsdm_free_fn rel = nullptr;       // null: hipFree
  void* rel_ctx = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  void alloc(size_t nbytes);
  void release();
  void upload(const void* host, size_t nbytes);
  void swap(DevBuf& o) {              // exchange buffers with their release functions
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
    std::swap(rel, o.rel);
    std::swap(rel_ctx, o.rel_ctx);
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// image (n0, n1, n2), each in [-128, 127], packed as offset binary so that the
// packed integer orders lexicographically like the triple
__host__ __device__ inline i32 img_pack(int n0, int n1, int n2) {
  return ((n0 + 128) << 16) | ((n1 + 128) << 8) | (n2 + 128);
}

// Squared distance of a pair for the range test: d = x_j - x_i (+ the lattice
// translation m T when periodic), with explicit fused multiply-adds so that
// the host search and the GPU search decide every pair (r^2 <= R^2, inclusive)
// the same way.
__host__ __device__ inline double pair_dist2(const double* xi, const double* xj, int m0, int m1, int m2,
                                             const double* T) {
  double dx = xj[0] - xi[0], dy = xj[1] - xi[1], dz = xj[2] - xi[2];
  if (T) {
    dx += fma((double)m2, T[6], fma((double)m1, T[3], (double)m0 * T[0]));
    dy += fma((double)m2, T[7], fma((double)m1, T[4], (double)m0 * T[1]));
    dz += fma((double)m2, T[8], fma((double)m1, T[5], (double)m0 * T[2]));
  }
  return fma(dz, dz, fma(dy, dy, dx * dx));
}
__host__ __device__ inline int img_c0(i32 p) { return ((p >> 16) & 255) - 128; }
__host__ __device__ inline int img_c1(i32 p) { return ((p >> 8) & 255) - 128; }
__host__ __device__ inline int img_c2(i32 p) { return (p & 255) - 128; }
__host__ __device__ inline i32 img_add(i32 a, i32 b) {  // a + b on unpacked triples
  return (((img_c0(a) + img_c0(b)) + 128) << 16) | (((img_c1(a) + img_c1(b)) + 128) << 8) | ((img_c2(a) + img_c2(b)) + 128);
}
__host__ __device__ inline i32 img_neg(i32 a) {
  return ((-img_c0(a) + 128) << 16) | ((-img_c1(a) + 128) << 8) | (-img_c2(a) + 128);
}
constexpr i32 IMG0 = (128 << 16) | (128 << 8) | 128;
// strip key: column quad and image in one sortable 64-bit value
__host__ __device__ inline i64 skey(i32 quad, i32 img) { return ((i64)quad << 24) | (i64)img; }
// Half of a symmetric matrix that a half-output product computes: strips
// whose column quad lies above the row's quad, and the row's own quad at
// images >= 0.  The other strips are mirrors of these: block (p, q, n) of a
// dropped strip is the transpose of (q, p, -n), which lies in a kept strip.
__host__ __device__ inline bool keep_strip(i32 row, i32 quad, i32 img) {
  return quad > (row >> 2) || (quad == (row >> 2) && img >= IMG0);
}

}  // namespace lsdm

// -------- handles ------------------------------------------------------------
struct lsdm_system {
  int device = 0;
  lsdm::i32 n_atoms = 0;
  std::vector<double> xyz;          // user order, 3 per atom
  std::vector<lsdm::i32> nfn;       // user order
  bool periodic = false;
  double lat[9] = {0}, inv[9] = {0};
  // Hilbert ordering and pseudo-atoms
  std::vector<lsdm::i32> order;     // internal atom position -> user atom
  std::vector<lsdm::i32> pbase;     // user atom -> first pseudo-atom
  std::vector<lsdm::i32> npseudo;   // user atom -> number of pseudo-atoms
  std::vector<lsdm::i32> patom;     // pseudo-atom -> user atom
  std::vector<lsdm::i32> prows;     // pseudo-atom -> real rows (1..4)
  std::vector<uint8_t> first;       // pseudo-atom -> 1 if first of its atom
  lsdm::i32 n_pseudo = 0;           // padded to a multiple of 4
  lsdm::i32 n_quads = 0;
  lsdm::DevBuf d_prows;             // i32[n_pseudo]
  lsdm::DevBuf d_first;             // u8[n_pseudo]
  lsdm::DevBuf d_patom;             // i32[n_pseudo], -1 for padding
  lsdm::DevBuf d_pbase, d_npseudo;  // i32[n_atoms] (user atom -> first pseudo-atom, count)
};

struct lsdm_pattern {
  const lsdm_system* sys = nullptr;
  double R = 0;
  // block layout (user), host
  std::vector<lsdm::i64> row_ptr;   // n_atoms + 1
  std::vector<lsdm::i32> col;       // user atom j
  std::vector<lsdm::i32> img;       // packed image
  std::vector<lsdm::i64> val_off;
  lsdm::i64 nval = 0;
  // strip layout, host
  std::vector<lsdm::i64> sptr;      // n_pseudo + 1
  std::vector<lsdm::i32> squad;     // column quad
  std::vector<lsdm::i32> simg;      // packed image
  std::vector<uint8_t> smask;       // 4-bit block mask
  lsdm::i64 n_strips = 0;
  // device copies
  lsdm::DevBuf d_sptr, d_squad, d_simg, d_smask;
  lsdm::DevBuf d_srow;              // i32 per strip: its row (pseudo-atom)
  // block layout <-> strip layout map: one entry per 4x4 sub-block of every
  // user block: user value offset of the sub-block's (0,0) element, its
  // strip-layout offset, and its real extent (rows, cols, user row stride)
  lsdm::i64 n_sub = 0;
  lsdm::DevBuf d_sub_user, d_sub_strip, d_sub_shape;   // i64, i64, i32 (rows | cols<<8 | stride<<16)
  // mirror map for transposes in strip layout: for strip s of row p, the
  // strip index of (q, quad(p), -n) for each of its 4 blocks q
  lsdm::DevBuf d_mirror;            // i64[4 * n_strips], -1 when absent
  // blocks that a symmetric result takes from their mirrors: strip index << 4
  // | mask of its blocks to fill (strips outside keep_strip, and the blocks
  // below the diagonal in a row's own quad at image 0)
  lsdm::i64 n_fill = 0;
  lsdm::DevBuf d_fill;
  bool maps_ready = false;          // the maps above are built on first use
  // writes of a symmetric result's half-output product, one i32 per block
  // slot of every kept strip: bit 0 set when the block is written in place
  // (clear for a present block below the diagonal in its row's own quad at
  // image 0, which is written as the mirror of the block above), bits 1..31
  // the mirror block's index + 1 when the product also writes that mirror
  // (its transpose) into the dropped half, else 0.  Built on first use.
  lsdm::DevBuf d_mirw;
  bool mirw_ready = false;
  // partial sums of lsdm_dot (allocated on its first call)
  lsdm::DevBuf d_dotpart;
  std::mutex maps_mutex;
};

namespace lsdm {

// Group tiles of the product kernels: a workgroup of GQ wavefronts computes
// GQ consecutive row quads (4 * GQ output rows, one quad per wavefront) x GJ
// column quads over one shared step list, the union of the rows' inner
// entries, so every B strip of a step is fetched once for all GQ row quads.
constexpr int GQ = 4;
constexpr int GJ = 8;
constexpr int GROWS = 4 * GQ;
// groups per super-group of the tile traversal order
#ifndef LSDM_GSUPER
#define LSDM_GSUPER 4
#endif
constexpr int GSUPER = LSDM_GSUPER;

struct GTile {
  i32 group;            // rows 4*GQ*group .. +4*GQ-1
  i32 nsteps;
  i64 step0;
  i32 cstrip[GROWS * GJ];   // output strip of slot (row r, jq) = [GJ*r + jq], -1 if absent
};

// One step of a group tile (128 bytes):
//   a[r]: strip-layout offset / 16 of A_{r,k} (X_{k,r} for a transposed A), -1 if absent
//   b[jq]: strip index of B's strip (k, quad jq), -1 if absent
//   mask[w]: slots of wavefront w, bit GJ*i + jq for row 4w+i
//   rows: bit r set when a[r] >= 0
//   bcols: bit jq set when b[jq] >= 0
struct alignas(128) GStep {
  i32 a[GROWS];
  i32 b[GJ];
  uint32_t mask[GQ];
  uint32_t rows;
  uint32_t bcols;
  i32 pad[2];
};
static_assert(sizeof(GStep) == 128, "group step record is 128 bytes");
static_assert(4 * GJ <= 32, "a wavefront's slots fit one 32-bit mask");

}  // namespace lsdm

struct lsdm_plan {
  const lsdm_pattern* A = nullptr;
  const lsdm_pattern* B = nullptr;
  const lsdm_pattern* C = nullptr;
  int transA = 0, transB = 0;
  int half = 0;                     // output restricted to keep_strip (symmetric result)
  lsdm::i64 n_triples = 0;
  double flops = 0;
  // group tiles and their steps
  lsdm::i64 n_gtiles = 0, n_gsteps = 0;
  lsdm::DevBuf d_gtiles, d_gsteps;
  lsdm::DevBuf d_queue;             // per-XCD tile counters of the product kernels (8 x u64)
  // residual mode (built on first use): for every output block, the B blocks
  // (p', q, n) with p' in p's atom and the op(A) blocks (p, q', n) with q' in
  // q's atom (rc_np per block, block index = value offset / 16, -1 if absent);
  // per pseudo-atom the on-site blocks op(A)_{p,p',0} and B_{q',q,0}
  int rc_np = 0;
  lsdm::DevBuf d_rc_b, d_rc_a, d_rc_aon, d_rc_bon;
  bool rc_ready = false;
  std::mutex rc_mutex;
  // for a transposed B the plan multiplies by a materialised transpose
  lsdm::DevBuf d_bT;                // strip-layout workspace of B^T (doubles)
  // stand-alone multiplies: strip-layout workspaces of the operands (grown on
  // first use in a precision, then kept), and the two plans of the adjoint
  // (built on first use), so repeated calls allocate and plan nothing
  lsdm::DevBuf mw[8];
  std::mutex mw_mutex;
  lsdm_plan* adjA = nullptr;        // plan of Abar += P_A(...)
  lsdm_plan* adjB = nullptr;        // plan of Bbar += P_B(...)
  std::mutex adj_mutex;
  ~lsdm_plan();
};

struct lsdm_lnv {
  const lsdm_system* sys = nullptr;
  double rS = 0, rH = 0, rL = 0;
  // symmetric mode: L, S, H are symmetric, so M and P are computed on one
  // half (F2, F3 half-output plans) and mirrored, and the adjoint takes dE/dL
  // as V + V^T - 4 X^T Y with Y = HX on M's range (B1), the last term a
  // half-output product (B3), V = 6 Y on L plus Xbar S (B5); B4 is null
  bool sym = false;
  lsdm_pattern *pS = nullptr, *pH = nullptr, *pL = nullptr, *pX = nullptr, *pM = nullptr;
  lsdm_plan *F1 = nullptr, *F2 = nullptr, *F3 = nullptr;
  lsdm_plan *B1 = nullptr, *B2 = nullptr, *B3 = nullptr, *B4 = nullptr, *B5 = nullptr;
  lsdm::i64 max_strips = 0;
  // strip-layout workspaces (sized for FP64)
  lsdm::DevBuf wL, wS, wH, wH64, wX, wM, wP, wMb, wXb, wLb, wK;
  lsdm::DevBuf wV;                  // symmetric mode: V = 6 H X - 4 H M S on L's pattern
  // symmetric mode: F2 writes M's dropped half as mirrors of the kept one
  // and leaves the absent blocks of dropped strips alone, which F3 and B2
  // read as zero.  wM_zero is the element size (4 or 8) for which wM was
  // zeroed and since written only that way; 0 after any other writer
  int wM_zero = 0;
  lsdm::DevBuf wE;                  // partial sums for the energy
  // map from H's strips to M's strips (K assembly and 6H into Mbar)
  lsdm::DevBuf d_h2m;               // i64 per H strip: M strip index (-1: none)
  lsdm::DevBuf d_mneed;             // u8 per M strip: 1 when some H strip maps to it
  lsdm::DevBuf d_l2y;               // symmetric mode: i64 per L strip, the M strip of Y = HX to project
  lsdm::DevBuf d_yneed;             // symmetric mode: u8 per M strip, 1 when an L strip maps to it
  // bf16 operand copies (allocated on first BF16 use): R = row-major blocks,
  // C = block-transposed; L_R L_C S_C H_R H_C X_R X_C M_C Mb_R Mb_C Xb_R
  lsdm::DevBuf b16[11];
  bool b16_ready = false;
  // residual mode: fp32 copies of the off-site parts (L S H X M Mb Xb) and the
  // fp32 product of the off-site parts
  lsdm::DevBuf r32[7], rr32;
  bool rc_ready = false;
  // S's blocks inside H's pattern (built on first use): per S block its value
  // offset, the value offset of the same block in H, and its size
  lsdm::i64 n_sblk = 0;
  lsdm::DevBuf d_s2h_s, d_s2h_h, d_s2h_n;
  bool s2h_ready = false;
  std::mutex s2h_mutex;
  lsdm::DevBuf wSh;                 // S on H's pattern (electron count)
  // McWeeny step on L's range (built on first use): LSL on 2 rL + rS (pM2,
  // or M itself when its range is that large), LSLSL on L's range, and the
  // map from L's strips to pM2's strips
  lsdm_pattern* pM2 = nullptr;      // owned only when distinct from pM
  lsdm_plan *P2 = nullptr, *P3 = nullptr;   // P2 null when F2 serves
  lsdm::DevBuf d_l2m, wM2, wP2, wK2;
  bool pur_ready = false;
  std::mutex pur_mutex;
  // optional kernel timing: event pairs around product launches
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_prod;         // product index 0..7 of each recorded pair
  ~lsdm_lnv();
};
