// C ABI of the lsdm library (declared in include/lsdm.h).
//
// The LNV chain (Bowler & Miyazaki, eq. 3 and the energy 2 Tr(KH)):
//   forward   F1  X = P_X(L S)        X on R_L + R_S
//             F2  M = P_M(X L)        M on min(2 R_L + R_S, R_H + R_L + R_S)
//             F3  P = P_H(X M)        (= LSLSL on H's range)
//             K = 3 M|_H - 2 P,  E = 2 <K, H>
//   adjoint   Kbar = 2H, Pbar = -4H
//             B1  Mbar = 6H + P_M(X^T Pbar)
//             B2  Xbar = P_X(Pbar M)
//             B3  Xbar += P_X(Mbar L)
//             B4  Lbar = P_L(X^T Mbar)
//             B5  Lbar += P_L(Xbar S)
// Taking LSLSL as X M = (LS)(LSL) keeps the chain equal to eq. 3 for any L, so
// the adjoint yields dE/dL of eq. 3 itself: 6 (HLS + SLH) - 4 (HLSLS + SLHLS + SLSLH).
// Symmetric mode (S, H, L symmetric, so Xᵀ = SL and M = LSL are known
// transposes) groups the same terms as dE/dL = V + Vᵀ - 4 XᵀHX with
// V = 6 HX - 4 HMS, each on L's range, and forms HX once:
//             B1  Y    = P_M(H X)
//             B2  Xbar = P_X(Pbar M)              (= -4 HM)
//             B3  Lbar = -4 P_L(X^T Y)            (= -4 XᵀHX, symmetric: half)
//             B4  V    = 6 P_L(Y)                 (a projection, no product)
//             B5  V   += P_L(Xbar S)
//             Lbar += V + Vᵀ, then the dropped half is mirrored.
// Every truncation keeps what L's range reaches: X's range holds all of
// P_X(HM) that (HM)S needs on L, and M's range all of HX (nonzero within
// R_H + R_X) that Xᵀ(HX) needs on L, so the regrouped chain equals the one
// above up to rounding.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <type_traits>

#include "kernels.h"
#include "lsdm_internal.h"

namespace lsdm {
void build_system(lsdm_system* s);
void build_pattern_blocks(lsdm_pattern* p);
void build_pattern_reach(lsdm_pattern* p, const lsdm_pattern* A, const lsdm_pattern* B);
void build_strips(lsdm_pattern* p);
void build_plan(lsdm_plan* pl);

static thread_local std::string g_last_error;
void set_error(int code, const std::string& msg) {
  (void)code;
  g_last_error = msg;
}

// Without a HIP device the symbolic pass still runs on the host (patterns,
// plans and their counts can be built and inspected) but device buffers stay
// empty and every compute call fails with LSDM_EDEVICE.
bool have_device() {
  static int state = -1;
  if (state < 0) {
    int n = 0;
    state = (hipGetDeviceCount(&n) == hipSuccess && n > 0) ? 1 : 0;
    (void)hipGetLastError();
  }
  return state == 1;
}
static void require_device() {
  if (!have_device()) LSDM_THROW(LSDM_EDEVICE, "no HIP device: compute calls need an MI355X (gfx950)");
}

// the caller's workspace allocator (lsdm_set_allocator); null: hipMalloc
static std::mutex g_alloc_mu;
static lsdm_alloc_fn g_alloc = nullptr;
static lsdm_free_fn g_free = nullptr;
static void* g_alloc_ctx = nullptr;

DevBuf::~DevBuf() {
  if (!p) return;
  if (rel) rel(p, rel_ctx);
  else (void)hipFree(p);
}
void DevBuf::release() {
  if (!p) return;
  void* q = p;
  p = nullptr;
  bytes = 0;
  if (rel) rel(q, rel_ctx);
  else HIP_CHECK(hipFree(q));
}
void DevBuf::alloc(size_t nbytes) {
  release();
  if (nbytes == 0) nbytes = 16;
  if (!have_device()) return;
  lsdm_alloc_fn a;
  lsdm_free_fn f;
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
    f = g_free;
    ctx = g_alloc_ctx;
  }
  if (a) {
    void* q = a(nbytes, ctx);
    if (!q) LSDM_THROW(LSDM_ENOMEM, "the caller's allocator returned NULL for " + std::to_string(nbytes) + " bytes");
    if (reinterpret_cast<uintptr_t>(q) & 255u) {
      f(q, ctx);
      LSDM_THROW(LSDM_EINVAL, "the caller's allocator returned memory not aligned to 256 bytes");
    }
    p = q;
    rel = f;
    rel_ctx = ctx;
  } else {
    HIP_CHECK(hipMalloc(&p, nbytes));
    rel = nullptr;
    rel_ctx = nullptr;
  }
  bytes = nbytes;
}
void DevBuf::upload(const void* host, size_t nbytes) {
  alloc(nbytes);
  if (nbytes && p) HIP_CHECK(hipMemcpy(p, host, nbytes, hipMemcpyHostToDevice));
}

template <class F>
static int guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return LSDM_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return LSDM_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return LSDM_EDEVICE;
  }
}

static void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) LSDM_THROW(LSDM_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

static lsdm_pattern* make_pattern(const lsdm_system* sys, double R) {
  if (!(R >= 0.0) || !std::isfinite(R)) LSDM_THROW(LSDM_EINVAL, "range must be finite and >= 0");
  std::unique_ptr<lsdm_pattern> p(new lsdm_pattern());
  p->sys = sys;
  p->R = R;
  build_pattern_blocks(p.get());
  build_strips(p.get());
  return p.release();
}

// the blocks of the sphere of R that a product of A's and B's patterns reaches
static lsdm_pattern* make_reach_pattern(const lsdm_system* sys, double R, const lsdm_pattern* A,
                                        const lsdm_pattern* B) {
  std::unique_ptr<lsdm_pattern> p(new lsdm_pattern());
  p->sys = sys;
  p->R = R;
  build_pattern_reach(p.get(), A, B);
  build_strips(p.get());
  return p.release();
}

static lsdm_plan* make_plan(const lsdm_pattern* A, int tA, const lsdm_pattern* B, int tB, const lsdm_pattern* C,
                            bool half = false) {
  if (!A || !B || !C) LSDM_THROW(LSDM_EINVAL, "null pattern");
  if (A->sys != B->sys || A->sys != C->sys) LSDM_THROW(LSDM_EPATTERN, "patterns belong to different systems");
  std::unique_ptr<lsdm_plan> pl(new lsdm_plan());
  pl->A = A;
  pl->B = B;
  pl->C = C;
  pl->transA = tA ? 1 : 0;
  pl->transB = tB ? 1 : 0;
  pl->half = half ? 1 : 0;
  build_plan(pl.get());
  return pl.release();
}

static size_t strip_bytes(const lsdm_pattern* p, size_t elem) { return (size_t)p->n_strips * 64 * elem + 64; }

// Workspace slot k of a plan's stand-alone multiplies, at least `bytes` long:
// allocated on first use and grown when a wider precision needs more, then
// kept with the plan (calls on one plan are ordered on their stream, so the
// same buffers serve every call).
enum { MW_A, MW_B, MW_BT, MW_C, MW_A2, MW_B2, MW_C2 };
template <class T>
static T* plan_ws(const lsdm_plan* cpl, int k, const lsdm_pattern* p, size_t elem) {
  lsdm_plan* pl = const_cast<lsdm_plan*>(cpl);
  std::lock_guard<std::mutex> g(pl->mw_mutex);
  const size_t need = strip_bytes(p, elem);
  if (pl->mw[k].bytes < need) pl->mw[k].alloc(need);
  return pl->mw[k].as<T>();
}

template <class T>
static void multiply_t(const lsdm_plan* pl, double alpha, const double* dA, const double* dB, double beta, double* dC,
                       hipStream_t st) {
  T* a = plan_ws<T>(pl, MW_A, pl->A, sizeof(T));
  T* b = plan_ws<T>(pl, MW_B, pl->B, sizeof(T));
  T* c = plan_ws<T>(pl, MW_C, pl->C, sizeof(T));
  fill<T>(a, pl->A->n_strips * 64, (T)0, st);
  fill<T>(b, pl->B->n_strips * 64, (T)0, st);
  fill<T>(c, pl->C->n_strips * 64, (T)0, st);
  user_to_strip<T>(pl->A, dA, a, 1.0, st);
  user_to_strip<T>(pl->B, dB, b, 1.0, st);
  const T* Bop = b;
  if (pl->transB) {
    T* bt = plan_ws<T>(pl, MW_BT, pl->B, sizeof(T));
    transpose_strips<T>(pl->B, b, bt, st);
    Bop = bt;
  }
  if (beta != 0.0) user_to_strip<T>(pl->C, dC, c, 1.0, st);
  product<T>(pl, a, Bop, c, alpha, beta, st);
  strip_to_user<T>(pl->C, c, dC, st);
  check_launch();
}

static void multiply_bf16(const lsdm_plan* pl, double alpha, const double* dA, const double* dB, double beta,
                          double* dC, hipStream_t st) {
  typedef unsigned short u16;
  float* a32 = plan_ws<float>(pl, MW_A, pl->A, 4);
  float* b32 = plan_ws<float>(pl, MW_B, pl->B, 4);
  float* c32 = plan_ws<float>(pl, MW_C, pl->C, 4);
  u16* a16 = plan_ws<u16>(pl, MW_A2, pl->A, 2);
  u16* b16 = plan_ws<u16>(pl, MW_B2, pl->B, 2);
  fill<float>(a32, pl->A->n_strips * 64, 0.f, st);
  fill<float>(b32, pl->B->n_strips * 64, 0.f, st);
  fill<float>(c32, pl->C->n_strips * 64, 0.f, st);
  user_to_strip<float>(pl->A, dA, a32, 1.0, st);
  user_to_strip<float>(pl->B, dB, b32, 1.0, st);
  // A: row-major copy, or for a transposed A the block-transposed copy of A
  to_bf16(a32, pl->transA ? nullptr : a16, pl->transA ? a16 : nullptr, pl->A->n_strips * 64, st);
  const float* bsrc = b32;
  if (pl->transB) {
    float* bt32 = plan_ws<float>(pl, MW_BT, pl->B, 4);
    transpose_strips<float>(pl->B, b32, bt32, st);
    bsrc = bt32;
  }
  to_bf16(bsrc, nullptr, b16, pl->B->n_strips * 64, st);
  if (beta != 0.0) user_to_strip<float>(pl->C, dC, c32, 1.0, st);
  product_bf16(pl, a16, b16, c32, alpha, beta, st);
  strip_to_user<float>(pl->C, c32, dC, st);
  check_launch();
}

// residual mode: FP64 master strips; FP32 product of the off-site parts; FP64
// block-diagonal correction
static void multiply_rc(const lsdm_plan* pl, double alpha, const double* dA, const double* dB, double beta, double* dC,
                        hipStream_t st) {
  double* a64 = plan_ws<double>(pl, MW_A, pl->A, 8);
  double* b64 = plan_ws<double>(pl, MW_B, pl->B, 8);
  double* c64 = plan_ws<double>(pl, MW_C, pl->C, 8);
  float* a32 = plan_ws<float>(pl, MW_A2, pl->A, 4);
  float* b32 = plan_ws<float>(pl, MW_B2, pl->B, 4);
  float* rr = plan_ws<float>(pl, MW_C2, pl->C, 4);
  fill<double>(a64, pl->A->n_strips * 64, 0.0, st);
  fill<double>(b64, pl->B->n_strips * 64, 0.0, st);
  fill<double>(c64, pl->C->n_strips * 64, 0.0, st);
  user_to_strip<double>(pl->A, dA, a64, 1.0, st);
  user_to_strip<double>(pl->B, dB, b64, 1.0, st);
  const double* bsrc = b64;
  if (pl->transB) {
    double* bt64 = plan_ws<double>(pl, MW_BT, pl->B, 8);
    transpose_strips<double>(pl->B, b64, bt64, st);
    bsrc = bt64;
  }
  offsite_f32(pl->A, a64, a32, st);
  offsite_f32(pl->B, bsrc, b32, st);
  if (beta != 0.0) user_to_strip<double>(pl->C, dC, c64, 1.0, st);
  product<float>(pl, a32, b32, rr, 1.0, 0.0, st);
  rc_correct(pl, a64, bsrc, rr, c64, alpha, beta, st);
  strip_to_user<double>(pl->C, c64, dC, st);
  check_launch();
}

// ---------------------------------------------------------------------------
// the LNV chain
// ---------------------------------------------------------------------------
// for every strip of `from`, the strip of `to` with the same (row, column
// quad, image); a strip `to` lacks maps to -1 when `what` is null, else it is
// an error (`to` must contain `from`)
static std::vector<i64> strip_map(const lsdm_system* sys, const lsdm_pattern* from, const lsdm_pattern* to,
                                  const char* what) {
  std::vector<i64> map(from->n_strips, -1);
  for (i32 q = 0; q < sys->n_pseudo; ++q) {
    i64 m = to->sptr[q];
    for (i64 h = from->sptr[q]; h < from->sptr[q + 1]; ++h) {
      const i64 key = skey(from->squad[h], from->simg[h]);
      while (m < to->sptr[q + 1] && skey(to->squad[m], to->simg[m]) < key) ++m;
      if (m >= to->sptr[q + 1] || skey(to->squad[m], to->simg[m]) != key) {
        if (what) LSDM_THROW(LSDM_EPATTERN, what);
        continue;
      }
      map[h] = m;
    }
  }
  return map;
}

static void lnv_build(lsdm_lnv* L) {
  const double rS = L->rS, rH = L->rH, rL = L->rL;
  const double rX = rL + rS, rM = std::min(2 * rL + rS, rH + rL + rS);
  L->pS = make_pattern(L->sys, rS);
  L->pH = make_pattern(L->sys, rH);
  L->pL = make_pattern(L->sys, rL);
  // X = LS is zero outside the blocks L S (or S L) reaches: on a crystal a
  // fifth of the rL + rS sphere (pairs no lattice path of an L step and an S
  // step connects), which every product that reads or writes X then skips
  L->pX = make_reach_pattern(L->sys, rX, L->pL, L->pS);
  L->pM = make_pattern(L->sys, rM);
  L->F1 = make_plan(L->pL, 0, L->pS, 0, L->pX);
  // symmetric mode: M = LSL, P = LSLSL and XᵀHX are symmetric, so their
  // products (F2, F3, B3 of the regrouped adjoint) fill one half
  const bool h = L->sym;
  L->F2 = make_plan(L->pX, 0, L->pL, 0, L->pM, h);
  L->F3 = make_plan(L->pX, 0, L->pM, 0, L->pH, h);
  // B1: Mbar = X^T Pbar on M's range, or in symmetric mode Y = H X there
  L->B1 = h ? make_plan(L->pH, 0, L->pX, 0, L->pM) : make_plan(L->pX, 1, L->pH, 0, L->pM);
  L->B2 = make_plan(L->pH, 0, L->pM, 0, L->pX);
  if (h) {
    L->B3 = make_plan(L->pX, 1, L->pM, 0, L->pL, true);    // X^T Y, half
    L->B4 = nullptr;                                        // V = 6 P_L(Y): a projection
  } else {
    L->B3 = make_plan(L->pM, 0, L->pL, 0, L->pX);
    L->B4 = make_plan(L->pX, 1, L->pM, 0, L->pL);
  }
  L->B5 = make_plan(L->pX, 0, L->pS, 0, L->pL);
  // H strip -> M strip with the same (row, column quad, image), -1 where M
  // has none: when rH > 2 rL + rS, LSL is zero beyond its own range, so those
  // blocks of K are -2 P alone and carry no 6H into Mbar
  const std::vector<i64> h2m = strip_map(L->sys, L->pH, L->pM, nullptr);
  L->d_h2m.upload(h2m.data(), sizeof(i64) * h2m.size());
  {   // M strips that K reads (the BF16 chain writes FP32 M only there)
    std::vector<uint8_t> need((size_t)L->pM->n_strips, 0);
    for (const i64 m : h2m)
      if (m >= 0) need[(size_t)m] = 1;
    L->d_mneed.upload(need.data(), need.size());
  }
  if (h) {   // L strip -> M strip (Y's projection on L's range; M's range holds L's)
    const std::vector<i64> l2y = strip_map(L->sys, L->pL, L->pM, "L range exceeds the LSL range");
    L->d_l2y.upload(l2y.data(), sizeof(i64) * l2y.size());
    std::vector<uint8_t> need((size_t)L->pM->n_strips, 0);   // M strips the projection reads
    for (const i64 m : l2y)
      if (m >= 0) need[(size_t)m] = 1;
    L->d_yneed.upload(need.data(), need.size());
  }
  auto ws = [](DevBuf& b, const lsdm_pattern* p) { b.alloc(strip_bytes(p, sizeof(double))); };
  ws(L->wL, L->pL);
  ws(L->wS, L->pS);
  ws(L->wH, L->pH);
  ws(L->wH64, L->pH);
  ws(L->wX, L->pX);
  ws(L->wM, L->pM);
  ws(L->wP, L->pH);
  ws(L->wK, L->pH);
  ws(L->wMb, L->pM);
  ws(L->wXb, L->pX);
  ws(L->wLb, L->pL);
  if (h) ws(L->wV, L->pL);
  L->wE.alloc(sizeof(double) * 4 * DOT_BLOCKS + 64);
}

// the chain's products in a fixed order: F1 F2 F3 B1 B2 B3 B4 B5
static lsdm_plan* chain_plan(const lsdm_lnv* L, int w) {
  lsdm_plan* p[8] = {L->F1, L->F2, L->F3, L->B1, L->B2, L->B3, L->B4, L->B5};
  return p[w];
}

template <class T>
static void chain_product(lsdm_lnv* L, int w, const T* A, const T* B, T* C, double alpha, double beta, hipStream_t st,
                          const T* Cin = nullptr, const i64* cmap = nullptr, bool mirrors = false) {
  if (!L->prof) {
    product<T>(chain_plan(L, w), A, B, C, alpha, beta, st, Cin, cmap, mirrors);
    return;
  }
  while (L->ev_pool.size() < L->ev_used + 2) {
    hipEvent_t e;
    HIP_CHECK(hipEventCreate(&e));
    L->ev_pool.push_back(e);
  }
  HIP_CHECK(hipEventRecord(L->ev_pool[L->ev_used], st));
  product<T>(chain_plan(L, w), A, B, C, alpha, beta, st, Cin, cmap, mirrors);
  HIP_CHECK(hipEventRecord(L->ev_pool[L->ev_used + 1], st));
  L->ev_used += 2;
  L->ev_prod.push_back(w);
}

// defer_p (symmetric mode, an energy-and-gradient call): P is not formed.
// Tr(PH) = Tr(XMH) = <X, HM> for symmetric M and H, and the adjoint forms
// Xbar = -4 P_X(HM) on X's pattern anyway, so E = 2 <3 M|_H, H> + <X, Xbar>:
// the forward pass leaves the partial sums of the first dot in wE and the
// backward pass adds the second after B2 and writes E.
template <class T>
static void lnv_forward(lsdm_lnv* L, const double* dL, const double* dS, const double* dH, double* dK, double* dE,
                        hipStream_t st, bool defer_p = false) {
  T* wL = L->wL.as<T>();
  T* wS = L->wS.as<T>();
  T* wH = L->wH.as<T>();
  T* wX = L->wX.as<T>();
  T* wM = L->wM.as<T>();
  T* wP = L->wP.as<T>();
  double* wH64 = L->wH64.as<double>();
  double* wK = L->wK.as<double>();
  // inputs into strip layout (padding and out-of-range blocks stay zero)
  fill<T>(wL, L->pL->n_strips * 64, (T)0, st);
  fill<T>(wS, L->pS->n_strips * 64, (T)0, st);
  fill<T>(wH, L->pH->n_strips * 64, (T)0, st);
  fill<double>(wH64, L->pH->n_strips * 64, 0.0, st);
  user_to_strip<T>(L->pL, dL, wL, 1.0, st);
  user_to_strip<T>(L->pS, dS, wS, 1.0, st);
  user_to_strip<T>(L->pH, dH, wH, 1.0, st);
  user_to_strip<double>(L->pH, dH, wH64, 1.0, st);
  chain_product<T>(L, 0, wL, wS, wX, 1.0, 0.0, st);     // X = LS
  if (L->sym && mirw_fits(L->pM)) {
    // M = XL on the kept half, the dropped half written as its mirrors
    if (L->wM_zero != (int)sizeof(T)) {
      fill<T>(wM, L->pM->n_strips * 64, (T)0, st);
      L->wM_zero = (int)sizeof(T);
    }
    chain_product<T>(L, 1, wX, wL, wM, 1.0, 0.0, st, nullptr, nullptr, true);
  } else {
    chain_product<T>(L, 1, wX, wL, wM, 1.0, 0.0, st);   // M = XL
    if (L->sym) {                                        // beyond the mirror words' reach: a fill pass
      sym_fill<T>(L->pM, wM, st);
      L->wM_zero = 0;
    }
  }
  if (defer_p) {
    kassembly<T>(L, wM, nullptr, wK, st);                                 // 3 M|_H
    dot_parts(wK, wH64, L->pH->n_strips * 64, L->wE.as<double>(), st);    // <3 M|_H, H>
    check_launch();
    return;
  }
  chain_product<T>(L, 2, wX, wM, wP, 1.0, 0.0, st);     // P = XM on H's range (kept half when symmetric)
  kassembly<T>(L, wM, wP, wK, st);                  // K = 3 M|_H - 2 P
  dot(wK, wH64, L->pH->n_strips * 64, 2.0, L->wE.as<double>(), dE, st);   // E = 2 <K, H>
  if (dK) strip_to_user<double>(L->pH, wK, dK, st);
  check_launch();
}

// dE: non-null when the forward pass deferred P (the energy is completed here)
template <class T>
static void lnv_backward(lsdm_lnv* L, double* dG, hipStream_t st, double* dE = nullptr) {
  T* wL = L->wL.as<T>();
  T* wS = L->wS.as<T>();
  T* wH = L->wH.as<T>();
  T* wX = L->wX.as<T>();
  T* wM = L->wM.as<T>();
  T* wMb = L->wMb.as<T>();
  T* wXb = L->wXb.as<T>();
  T* wLb = L->wLb.as<T>();
  if (!L->sym) {
    chain_product<T>(L, 3, wX, wH, wMb, -4.0, 0.0, st);  // Mbar = X^T Pbar,  Pbar = -4H (every M strip written)
    chain_product<T>(L, 4, wH, wM, wXb, -4.0, 0.0, st);  // Xbar  = Pbar M
    scatter_h<T>(L, wH, wMb, 6.0, st);                   // Mbar += 3 Kbar = 6H on H's range
    chain_product<T>(L, 5, wMb, wL, wXb, 1.0, 1.0, st);  // Xbar += Mbar L
    chain_product<T>(L, 6, wX, wMb, wLb, 1.0, 0.0, st);  // Lbar  = X^T Mbar
    chain_product<T>(L, 7, wXb, wS, wLb, 1.0, 1.0, st);  // Lbar += Xbar S
  } else {
    T* wV = L->wV.as<T>();
    T* wY = wMb;                                         // Y = H X on M's range (Mbar's workspace)
    chain_product<T>(L, 3, wH, wX, wY, 1.0, 0.0, st);    // Y = H X
    chain_product<T>(L, 4, wH, wM, wXb, -4.0, 0.0, st);  // Xbar = -4 H M
    if constexpr (std::is_same<T, double>::value) {
      if (dE) {                                          // E = 2 <3 M|_H, H> + <X, Xbar>
        dot_parts(wX, wXb, L->pX->n_strips * 64, L->wE.as<double>() + 2 * DOT_BLOCKS, st);
        dot_final2(L->wE.as<double>(), 2.0, 1.0, dE, st);
      }
    }
    chain_product<T>(L, 5, wX, wY, wLb, -4.0, 0.0, st);  // Lbar = -4 X^T Y = -4 X^T H X (half)
    // V = Xbar S + 6 P_L(Y) = -4 HMS + 6 HX on L: the projection of Y is B5's beta term
    chain_product<T>(L, 7, wXb, wS, wV, 1.0, 6.0, st, wY, L->d_l2y.as<i64>());
    sym_grad_to_user<T>(L->pL, wLb, wV, dG, st);         // dE/dL = Lbar + V + V^T, both halves
    check_launch();
    return;
  }
  strip_to_user<T>(L->pL, wLb, dG, st);
  check_launch();
}

// BF16 chain: bf16 operands, fp32 accumulation and fp32 master strips, K and E
// in FP64.  Intermediates are rounded to bf16 once, when they become operands.
enum { LR, LC, SC, HR, HC, XR, XC, MC, MbR, MbC, XbR };

// The copies are zeroed once when allocated: later writes touch only the
// pattern's elements (inputs) or whole strips (products, mirror fills), so
// padding and absent blocks stay zero.
static void bf16_workspaces(lsdm_lnv* L, hipStream_t st) {
  if (L->b16_ready) return;
  const lsdm_pattern* who[11] = {L->pL, L->pL, L->pS, L->pH, L->pH, L->pX, L->pX, L->pM, L->pM, L->pM, L->pX};
  for (int k = 0; k < 11; ++k) {
    L->b16[k].alloc(strip_bytes(who[k], 2));
    fill<unsigned short>(L->b16[k].as<unsigned short>(), (i64)(L->b16[k].bytes / 2), 0, st);
  }
  L->b16_ready = true;
}

static void chain_product_bf16(lsdm_lnv* L, int w, const unsigned short* A, const unsigned short* B, float* C,
                               double alpha, double beta, hipStream_t st, unsigned short* outR = nullptr,
                               unsigned short* outC = nullptr, const uint8_t* cneed = nullptr,
                               const float* Cin = nullptr, const i64* cmap = nullptr) {
  if (!L->prof) {
    product_bf16(chain_plan(L, w), A, B, C, alpha, beta, st, outR, outC, cneed, Cin, cmap);
    return;
  }
  while (L->ev_pool.size() < L->ev_used + 2) {
    hipEvent_t e;
    HIP_CHECK(hipEventCreate(&e));
    L->ev_pool.push_back(e);
  }
  HIP_CHECK(hipEventRecord(L->ev_pool[L->ev_used], st));
  product_bf16(chain_plan(L, w), A, B, C, alpha, beta, st, outR, outC, cneed, Cin, cmap);
  HIP_CHECK(hipEventRecord(L->ev_pool[L->ev_used + 1], st));
  L->ev_used += 2;
  L->ev_prod.push_back(w);
}

static void lnv_forward_bf16(lsdm_lnv* L, const double* dL, const double* dS, const double* dH, double* dK,
                             double* dE, hipStream_t st) {
  typedef unsigned short u16;
  bf16_workspaces(L, st);
  auto h = [&](int k) { return L->b16[k].as<u16>(); };
  float* wM = L->wM.as<float>();
  float* wP = L->wP.as<float>();
  double* wH64 = L->wH64.as<double>();
  double* wK = L->wK.as<double>();
  fill<double>(wH64, L->pH->n_strips * 64, 0.0, st);
  user_to_strip<double>(L->pH, dH, wH64, 1.0, st);
  // inputs straight from the caller's layout to their bf16 copies
  user_to_bf16(L->pL, dL, h(LR), h(LC), st);
  user_to_bf16(L->pS, dS, nullptr, h(SC), st);
  user_to_bf16(L->pH, dH, h(HR), h(HC), st);
  if (!L->sym) {                                               // FP32 H for Mbar += 6H
    float* wH = L->wH.as<float>();
    fill<float>(wH, L->pH->n_strips * 64, 0.f, st);
    user_to_strip<float>(L->pH, dH, wH, 1.0, st);
  }
  // X = LS: only its bf16 copies are used later
  chain_product_bf16(L, 0, h(LR), h(SC), nullptr, 1.0, 0.0, st, h(XR), h(XC));
  // M = XL: FP32 only on the strips K reads (kept half when symmetric: K
  // reads mirrors), and the block-transposed bf16 copy for the products,
  // whose epilogue writes the dropped half of a symmetric M as well (the copy
  // of a mirror block is the row-major copy of its kept block)
  chain_product_bf16(L, 1, h(XR), h(LC), wM, 1.0, 0.0, st, nullptr, h(MC), L->d_mneed.as<uint8_t>());
  L->wM_zero = 0;
  chain_product_bf16(L, 2, h(XR), h(MC), wP, 1.0, 0.0, st);    // P = XM on H's range
  kassembly<float>(L, wM, wP, wK, st);
  dot(wK, wH64, L->pH->n_strips * 64, 2.0, L->wE.as<double>(), dE, st);
  if (dK) strip_to_user<double>(L->pH, wK, dK, st);
  check_launch();
}

static void lnv_backward_bf16(lsdm_lnv* L, double* dG, hipStream_t st) {
  typedef unsigned short u16;
  auto h = [&](int k) { return L->b16[k].as<u16>(); };
  float* wH = L->wH.as<float>();
  float* wMb = L->wMb.as<float>();
  float* wXb = L->wXb.as<float>();
  float* wLb = L->wLb.as<float>();
  if (!L->sym) {
    chain_product_bf16(L, 3, h(XC), h(HC), wMb, -4.0, 0.0, st);   // Mbar = X^T Pbar
    scatter_h<float>(L, wH, wMb, 6.0, st);                          // Mbar += 6H
    to_bf16(wMb, h(MbR), h(MbC), L->pM->n_strips * 64, st);
    chain_product_bf16(L, 4, h(HR), h(MC), wXb, -4.0, 0.0, st);   // Xbar = Pbar M
    chain_product_bf16(L, 5, h(MbR), h(LC), wXb, 1.0, 1.0, st);   // Xbar += Mbar L
    to_bf16(wXb, h(XbR), nullptr, L->pX->n_strips * 64, st);
    chain_product_bf16(L, 6, h(XC), h(MbC), wLb, 1.0, 0.0, st);   // Lbar = X^T Mbar
    chain_product_bf16(L, 7, h(XbR), h(SC), wLb, 1.0, 1.0, st);   // Lbar += Xbar S
  } else {
    float* wV = L->wV.as<float>();
    float* wY = wMb;
    // Y = H X: FP32 for its projection, block-transposed bf16 copy as the
    // B operand of X^T Y (in Mbar's bf16 slot); Xbar is an operand only
    chain_product_bf16(L, 3, h(HR), h(XC), wY, 1.0, 0.0, st, nullptr, h(MbC),          // Y = H X (FP32 only
                       L->d_yneed.as<uint8_t>());                                       // on L's strips)
    chain_product_bf16(L, 4, h(HR), h(MC), nullptr, -4.0, 0.0, st, h(XbR), nullptr);   // Xbar = Pbar M
    chain_product_bf16(L, 5, h(XC), h(MbC), wLb, -4.0, 0.0, st); // Lbar = -4 X^T Y (half)
    chain_product_bf16(L, 7, h(XbR), h(SC), wV, 1.0, 6.0, st, nullptr, nullptr, nullptr,   // V = Xbar S
                       wY, L->d_l2y.as<i64>());                                               //   + 6 P_L(Y)
    sym_grad_to_user<float>(L->pL, wLb, wV, dG, st);              // dE/dL = Lbar + V + V^T
    check_launch();
    return;
  }
  strip_to_user<float>(L->pL, wLb, dG, st);
  check_launch();
}

// Residual chain: every intermediate in FP64; each product is the FP32 product
// of the off-site parts (timed as the chain's product) plus the FP64
// block-diagonal correction.
enum { RL, RS, RH, RX, RM, RMb, RXb };

static void rc_workspaces(lsdm_lnv* L) {
  if (L->rc_ready) return;
  const lsdm_pattern* who[7] = {L->pL, L->pS, L->pH, L->pX, L->pM, L->pM, L->pX};
  for (int k = 0; k < 7; ++k) L->r32[k].alloc(strip_bytes(who[k], 4));
  L->rr32.alloc(strip_bytes(L->pM, 4));
  L->rc_ready = true;
}

static void rc_step(lsdm_lnv* L, int w, const double* A64, const float* A32, const double* B64, const float* B32,
                    double* C64, double alpha, double beta, hipStream_t st) {
  float* rr = L->rr32.as<float>();
  chain_product<float>(L, w, A32, B32, rr, 1.0, 0.0, st);
  rc_correct(chain_plan(L, w), A64, B64, rr, C64, alpha, beta, st);
}

static void lnv_forward_rc(lsdm_lnv* L, const double* dL, const double* dS, const double* dH, double* dK, double* dE,
                           hipStream_t st) {
  rc_workspaces(L);
  auto r = [&](int k) { return L->r32[k].as<float>(); };
  double* wL = L->wL.as<double>();
  double* wS = L->wS.as<double>();
  double* wH = L->wH64.as<double>();
  double* wX = L->wX.as<double>();
  double* wM = L->wM.as<double>();
  double* wP = L->wP.as<double>();
  double* wK = L->wK.as<double>();
  fill<double>(wL, L->pL->n_strips * 64, 0.0, st);
  fill<double>(wS, L->pS->n_strips * 64, 0.0, st);
  fill<double>(wH, L->pH->n_strips * 64, 0.0, st);
  user_to_strip<double>(L->pL, dL, wL, 1.0, st);
  user_to_strip<double>(L->pS, dS, wS, 1.0, st);
  user_to_strip<double>(L->pH, dH, wH, 1.0, st);
  offsite_f32(L->pL, wL, r(RL), st);
  offsite_f32(L->pS, wS, r(RS), st);
  offsite_f32(L->pH, wH, r(RH), st);
  rc_step(L, 0, wL, r(RL), wS, r(RS), wX, 1.0, 0.0, st);       // X = LS
  offsite_f32(L->pX, wX, r(RX), st);
  rc_step(L, 1, wX, r(RX), wL, r(RL), wM, 1.0, 0.0, st);       // M = XL
  if (L->sym) sym_fill<double>(L->pM, wM, st);
  L->wM_zero = 0;
  offsite_f32(L->pM, wM, r(RM), st);
  rc_step(L, 2, wX, r(RX), wM, r(RM), wP, 1.0, 0.0, st);       // P = XM on H's range
  kassembly<double>(L, wM, wP, wK, st);
  dot(wK, wH, L->pH->n_strips * 64, 2.0, L->wE.as<double>(), dE, st);
  if (dK) strip_to_user<double>(L->pH, wK, dK, st);
  check_launch();
}

static void lnv_backward_rc(lsdm_lnv* L, double* dG, hipStream_t st) {
  auto r = [&](int k) { return L->r32[k].as<float>(); };
  double* wL = L->wL.as<double>();
  double* wS = L->wS.as<double>();
  double* wH = L->wH64.as<double>();
  double* wX = L->wX.as<double>();
  double* wM = L->wM.as<double>();
  double* wMb = L->wMb.as<double>();
  double* wXb = L->wXb.as<double>();
  double* wLb = L->wLb.as<double>();
  if (L->sym) rc_step(L, 3, wH, r(RH), wX, r(RX), wMb, 1.0, 0.0, st);   // Y = H X (in Mbar's workspace)
  else rc_step(L, 3, wX, r(RX), wH, r(RH), wMb, -4.0, 0.0, st);          // Mbar = X^T Pbar
  if (!L->sym) scatter_h<double>(L, wH, wMb, 6.0, st);         // Mbar += 6H
  offsite_f32(L->pM, wMb, r(RMb), st);
  rc_step(L, 4, wH, r(RH), wM, r(RM), wXb, -4.0, 0.0, st);     // Xbar = Pbar M
  if (!L->sym) {
    rc_step(L, 5, wMb, r(RMb), wL, r(RL), wXb, 1.0, 1.0, st);  // Xbar += Mbar L
    offsite_f32(L->pX, wXb, r(RXb), st);
    rc_step(L, 6, wX, r(RX), wMb, r(RMb), wLb, 1.0, 0.0, st);  // Lbar = X^T Mbar
    rc_step(L, 7, wXb, r(RXb), wS, r(RS), wLb, 1.0, 1.0, st);  // Lbar += Xbar S
  } else {
    double* wV = L->wV.as<double>();
    offsite_f32(L->pX, wXb, r(RXb), st);
    rc_step(L, 5, wX, r(RX), wMb, r(RMb), wLb, -4.0, 0.0, st); // Lbar = -4 X^T Y (half)
    project_strips<double>(L->pL, L->d_l2y.as<i64>(), wMb, wV, 6.0, st);   // V = 6 P_L(Y)
    rc_step(L, 7, wXb, r(RXb), wS, r(RS), wV, 1.0, 1.0, st);   // V += Xbar S
    sym_grad_to_user<double>(L->pL, wLb, wV, dG, st);            // dE/dL = Lbar + V + V^T
    check_launch();
    return;
  }
  strip_to_user<double>(L->pL, wLb, dG, st);
  check_launch();
}

// ---------------------------------------------------------------------------
// McWeeny step (section 2: eq. 3 as a map of L, which drives the eigenvalues
// of LS towards 0 and 1): L' = 3 LSL - 2 LSLSL on L's range.  LSLSL on L's
// range needs LSL on rL + rX = 2 rL + rS, more than the chain's M when
// rH < rL; that pattern and its plans are built on the first call.
// ---------------------------------------------------------------------------
static void purify_build(lsdm_lnv* L) {
  std::lock_guard<std::mutex> g(L->pur_mutex);
  if (L->pur_ready) return;
  const double rM2 = 2 * L->rL + L->rS;
  const double rM = std::min(2 * L->rL + L->rS, L->rH + L->rL + L->rS);
  const lsdm_pattern* M2 = L->pM;
  if (rM2 > rM) {
    L->pM2 = make_pattern(L->sys, rM2);
    L->P2 = make_plan(L->pX, 0, L->pL, 0, L->pM2);
    M2 = L->pM2;
    L->wM2.alloc(strip_bytes(M2, sizeof(double)));
  }
  L->P3 = make_plan(L->pX, 0, M2, 0, L->pL, L->sym);
  const std::vector<i64> l2m = strip_map(L->sys, L->pL, M2, "L range exceeds the LSL range");
  L->d_l2m.upload(l2m.data(), sizeof(i64) * l2m.size());
  L->wP2.alloc(strip_bytes(L->pL, sizeof(double)));
  L->wK2.alloc(strip_bytes(L->pL, sizeof(double)));
  L->pur_ready = true;
}

template <class T>
static void purify_chain(lsdm_lnv* L, const double* dL, const double* dS, double* dOut, hipStream_t st) {
  T* wL = L->wL.as<T>();
  T* wS = L->wS.as<T>();
  T* wX = L->wX.as<T>();
  const lsdm_pattern* M2 = L->pM2 ? L->pM2 : L->pM;
  T* wM2 = L->pM2 ? L->wM2.as<T>() : L->wM.as<T>();
  T* wP2 = L->wP2.as<T>();
  fill<T>(wL, L->pL->n_strips * 64, (T)0, st);
  fill<T>(wS, L->pS->n_strips * 64, (T)0, st);
  user_to_strip<T>(L->pL, dL, wL, 1.0, st);
  user_to_strip<T>(L->pS, dS, wS, 1.0, st);
  product<T>(L->F1, wL, wS, wX, 1.0, 0.0, st);                       // X = LS
  if (L->pM2) {
    product<T>(L->P2, wX, wL, wM2, 1.0, 0.0, st);                    // LSL on 2 rL + rS
  } else {
    product<T>(L->F2, wX, wL, wM2, 1.0, 0.0, st);                    // the chain's M suffices
    if (L->sym) sym_fill<T>(M2, wM2, st);
    L->wM_zero = 0;
  }
  product<T>(L->P3, wX, wM2, wP2, 1.0, 0.0, st);                     // LSLSL on L's range
  if (L->sym) sym_fill<T>(L->pL, wP2, st);
  kassembly_on<T>(L->pL, L->d_l2m.as<i64>(), wM2, wP2, L->wK2.as<double>(), st);   // 3 LSL - 2 LSLSL
  strip_to_user<double>(L->pL, L->wK2.as<double>(), dOut, st);
  check_launch();
}

}  // namespace lsdm

lsdm_plan::~lsdm_plan() {
  delete adjA;
  delete adjB;
}

lsdm_lnv::~lsdm_lnv() {
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
}

using namespace lsdm;

extern "C" {

int lsdm_set_allocator(lsdm_alloc_fn alloc, lsdm_free_fn release, void* ctx) {
  return guarded([&] {
    if ((alloc == nullptr) != (release == nullptr))
      LSDM_THROW(LSDM_EINVAL, "lsdm_set_allocator: alloc and release must both be set or both be NULL");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = alloc;
    g_free = release;
    g_alloc_ctx = alloc ? ctx : nullptr;
  });
}

const char* lsdm_last_error(void) { return g_last_error.c_str(); }
const char* lsdm_version(void) { return "lsdm 0.1 gfx950"; }

int lsdm_system_create(int32_t n_atoms, const double* xyz, const int32_t* nfn, const double* lattice,
                       lsdm_system** out) {
  return guarded([&] {
    if (!out || !xyz || !nfn || n_atoms <= 0) LSDM_THROW(LSDM_EINVAL, "null argument or n_atoms <= 0");
    *out = nullptr;
    std::unique_ptr<lsdm_system> s(new lsdm_system());
    if (have_device()) HIP_CHECK(hipGetDevice(&s->device));
    s->n_atoms = n_atoms;
    s->xyz.assign(xyz, xyz + 3 * (size_t)n_atoms);
    s->nfn.assign(nfn, nfn + n_atoms);
    for (double v : s->xyz)
      if (!std::isfinite(v)) LSDM_THROW(LSDM_EINVAL, "non-finite position");
    for (i32 v : s->nfn)
      if (v < 1 || v > 16) LSDM_THROW(LSDM_EINVAL, "nfn must lie in 1..16");
    if (lattice) {
      s->periodic = true;
      for (int k = 0; k < 9; ++k) {
        if (!std::isfinite(lattice[k])) LSDM_THROW(LSDM_EINVAL, "non-finite lattice");
        s->lat[k] = lattice[k];
      }
    }
    build_system(s.get());
    *out = s.release();
  });
}

void lsdm_system_destroy(lsdm_system* s) { delete s; }

int lsdm_pattern_create(const lsdm_system* sys, double range, lsdm_pattern** out) {
  return guarded([&] {
    if (!sys || !out) LSDM_THROW(LSDM_EINVAL, "null argument");
    *out = nullptr;
    *out = make_pattern(sys, range);
  });
}

int lsdm_pattern_info(const lsdm_pattern* p, int64_t* n_blocks, int64_t* n_values) {
  return guarded([&] {
    if (!p) LSDM_THROW(LSDM_EINVAL, "null pattern");
    if (n_blocks) *n_blocks = (int64_t)p->col.size();
    if (n_values) *n_values = p->nval;
  });
}

int lsdm_pattern_export(const lsdm_pattern* p, int64_t* row_ptr, int32_t* col, int8_t* img3, int64_t* val_off) {
  return guarded([&] {
    if (!p) LSDM_THROW(LSDM_EINVAL, "null pattern");
    if (row_ptr) std::memcpy(row_ptr, p->row_ptr.data(), sizeof(int64_t) * p->row_ptr.size());
    if (col) std::memcpy(col, p->col.data(), sizeof(int32_t) * p->col.size());
    if (val_off) std::memcpy(val_off, p->val_off.data(), sizeof(int64_t) * p->val_off.size());
    if (img3)
      for (size_t b = 0; b < p->img.size(); ++b) {
        img3[3 * b] = (int8_t)img_c0(p->img[b]);
        img3[3 * b + 1] = (int8_t)img_c1(p->img[b]);
        img3[3 * b + 2] = (int8_t)img_c2(p->img[b]);
      }
  });
}

void lsdm_pattern_destroy(lsdm_pattern* p) { delete p; }

int lsdm_plan_create(const lsdm_pattern* A, int transA, const lsdm_pattern* B, int transB, const lsdm_pattern* C,
                     lsdm_plan** out) {
  return guarded([&] {
    if (!out) LSDM_THROW(LSDM_EINVAL, "null argument");
    *out = nullptr;
    *out = make_plan(A, transA, B, transB, C);
  });
}

int lsdm_plan_info(const lsdm_plan* pl, int64_t* n_triples, double* flops, int64_t* plan_bytes) {
  return guarded([&] {
    if (!pl) LSDM_THROW(LSDM_EINVAL, "null plan");
    if (n_triples) *n_triples = pl->n_triples;
    if (flops) *flops = pl->flops;
    if (plan_bytes) *plan_bytes = (int64_t)(pl->n_gtiles * sizeof(GTile) + pl->n_gsteps * sizeof(GStep));
  });
}

void lsdm_plan_destroy(lsdm_plan* pl) { delete pl; }

int lsdm_multiply(const lsdm_plan* pl, int prec, double alpha, const double* dA, const double* dB, double beta,
                  double* dC, void* stream) {
  return guarded([&] {
    require_device();
    if (!pl || !dA || !dB || !dC) LSDM_THROW(LSDM_EINVAL, "null argument");
    if (dC == dA || dC == dB) LSDM_THROW(LSDM_EINVAL, "C must not alias A or B");
    hipStream_t st = (hipStream_t)stream;
    if (prec == LSDM_FP64) multiply_t<double>(pl, alpha, dA, dB, beta, dC, st);
    else if (prec == LSDM_FP32) multiply_t<float>(pl, alpha, dA, dB, beta, dC, st);
    else if (prec == LSDM_BF16) multiply_bf16(pl, alpha, dA, dB, beta, dC, st);
    else if (prec == LSDM_FP32_RC) multiply_rc(pl, alpha, dA, dB, beta, dC, st);
    else LSDM_THROW(LSDM_EINVAL, "unknown precision mode");
  });
}

int lsdm_multiply_adjoint(const lsdm_plan* pl, int prec, const double* dCbar, const double* dA, const double* dB,
                          double* dAbar, double* dBbar, void* stream) {
  return guarded([&] {
    require_device();
    if (!pl || !dCbar || !dA || !dB) LSDM_THROW(LSDM_EINVAL, "null argument");
    if (prec < LSDM_FP64 || prec > LSDM_FP32_RC) LSDM_THROW(LSDM_EINVAL, "unknown precision mode");
    hipStream_t st = (hipStream_t)stream;
    auto run = [&](const lsdm_plan* q, const double* x, const double* y, double* out) {
      if (prec == LSDM_FP64) multiply_t<double>(q, 1.0, x, y, 1.0, out, st);
      else if (prec == LSDM_FP32) multiply_t<float>(q, 1.0, x, y, 1.0, out, st);
      else if (prec == LSDM_BF16) multiply_bf16(q, 1.0, x, y, 1.0, out, st);
      else multiply_rc(q, 1.0, x, y, 1.0, out, st);
    };
    lsdm_plan* mp = const_cast<lsdm_plan*>(pl);
    if (dAbar) {
      // Abar += P_A(Cbar op(B)^T), or P_A(op(B) Cbar^T) when A enters transposed
      {
        std::lock_guard<std::mutex> g(mp->adj_mutex);
        if (!mp->adjA)
          mp->adjA = pl->transA ? make_plan(pl->B, pl->transB, pl->C, 1, pl->A)
                                : make_plan(pl->C, 0, pl->B, !pl->transB, pl->A);
      }
      if (pl->transA) run(mp->adjA, dB, dCbar, dAbar);
      else run(mp->adjA, dCbar, dB, dAbar);
    }
    if (dBbar) {
      // Bbar += P_B(op(A)^T Cbar), or P_B(Cbar^T op(A)) when B enters transposed
      {
        std::lock_guard<std::mutex> g(mp->adj_mutex);
        if (!mp->adjB)
          mp->adjB = pl->transB ? make_plan(pl->C, 1, pl->A, pl->transA, pl->B)
                                : make_plan(pl->A, !pl->transA, pl->C, 0, pl->B);
      }
      if (pl->transB) run(mp->adjB, dCbar, dA, dBbar);
      else run(mp->adjB, dA, dCbar, dBbar);
    }
  });
}

int lsdm_dot(const lsdm_pattern* p, const double* dA, const double* dB, double* dOut, void* stream) {
  return guarded([&] {
    require_device();
    if (!p || !dA || !dB || !dOut) LSDM_THROW(LSDM_EINVAL, "null argument");
    lsdm_pattern* q = const_cast<lsdm_pattern*>(p);
    {
      std::lock_guard<std::mutex> lk(q->maps_mutex);
      if (!q->d_dotpart.p) q->d_dotpart.alloc(sizeof(double) * 2 * DOT_BLOCKS);
    }
    dot(dA, dB, p->nval, 1.0, q->d_dotpart.as<double>(), dOut, (hipStream_t)stream);
    check_launch();
  });
}

int lsdm_dot_noalloc(const lsdm_pattern* p, const double* dA, const double* dB, double* dOut, void* stream) {
  return guarded([&] {
    require_device();
    if (!p || !dA || !dB || !dOut) LSDM_THROW(LSDM_EINVAL, "null argument");
    // the fixed grid needs DOT_SCRATCH partials whatever the pattern's size,
    // so every pattern fits the scratch
    static_assert(2 * DOT_BLOCKS <= DOT_SCRATCH, "dot partials exceed the scratch");
    double* part = dot_scratch();
    dot(dA, dB, p->nval, 1.0, part, dOut, (hipStream_t)stream);
    check_launch();
  });
}

int lsdm_lnv_create(const lsdm_system* sys, double rS, double rH, double rL, lsdm_lnv** out) {
  return lsdm_lnv_create_ex(sys, rS, rH, rL, 0, out);
}

int lsdm_lnv_create_ex(const lsdm_system* sys, double rS, double rH, double rL, int flags, lsdm_lnv** out) {
  return guarded([&] {
    if (!sys || !out) LSDM_THROW(LSDM_EINVAL, "null argument");
    *out = nullptr;
    if (flags & ~LSDM_LNV_SYMMETRIC) LSDM_THROW(LSDM_EINVAL, "unknown flag");
    for (double r : {rS, rH, rL})
      if (!(r >= 0.0) || !std::isfinite(r)) LSDM_THROW(LSDM_EINVAL, "ranges must be finite and >= 0");
    std::unique_ptr<lsdm_lnv> L(new lsdm_lnv());
    L->sys = sys;
    L->rS = rS;
    L->rH = rH;
    L->rL = rL;
    L->sym = (flags & LSDM_LNV_SYMMETRIC) != 0;
    try {
      lnv_build(L.get());
    } catch (...) {
      lsdm_lnv_destroy(L.release());
      throw;
    }
    *out = L.release();
  });
}

int lsdm_lnv_pattern(const lsdm_lnv* L, int which, const lsdm_pattern** out) {
  return guarded([&] {
    if (!L || !out) LSDM_THROW(LSDM_EINVAL, "null argument");
    const lsdm_pattern* ps[5] = {L->pS, L->pH, L->pL, L->pX, L->pM};
    if (which < 0 || which > 4) LSDM_THROW(LSDM_EINVAL, "which must be 0..4");
    *out = ps[which];
  });
}

int lsdm_lnv_info(const lsdm_lnv* L, int grad, int64_t* n_triples, double* flops) {
  return guarded([&] {
    if (!L) LSDM_THROW(LSDM_EINVAL, "null argument");
    const lsdm_plan* f[3] = {L->F1, L->F2, L->F3};
    const lsdm_plan* b[5] = {L->B1, L->B2, L->B3, L->B4, L->B5};
    int64_t nt = 0;
    double fl = 0;
    for (auto p : f) { nt += p->n_triples; fl += p->flops; }
    if (grad)
      for (auto p : b)
        if (p) { nt += p->n_triples; fl += p->flops; }
    if (n_triples) *n_triples = nt;
    if (flops) *flops = fl;
  });
}

// ---------------------------------------------------------------------------
// Minimisation of the LNV energy over L (the search the paper runs, section 2:
// the ground state is found by minimising E with respect to L).  Line search:
// E(L + tD) is a cubic polynomial of t (eq. 3 is cubic in L), so one line
// search is exact: its four coefficients come from four energies at
// t = -h, 0, h, 2h, and the step is the cubic's local minimum.  Directions:
// Polak-Ribiere conjugate gradients with restarts.
// ---------------------------------------------------------------------------
static void energy_any(lsdm_lnv* L, int prec, const double* dL, const double* dS, const double* dH, double* dE,
                       hipStream_t st) {
  if (prec == LSDM_FP64) lnv_forward<double>(L, dL, dS, dH, nullptr, dE, st);
  else if (prec == LSDM_FP32) lnv_forward<float>(L, dL, dS, dH, nullptr, dE, st);
  else if (prec == LSDM_BF16) lnv_forward_bf16(L, dL, dS, dH, nullptr, dE, st);
  else if (prec == LSDM_FP32_RC) lnv_forward_rc(L, dL, dS, dH, nullptr, dE, st);
  else LSDM_THROW(LSDM_EINVAL, "unknown precision mode");
}
static void energy_grad_any(lsdm_lnv* L, int prec, const double* dL, const double* dS, const double* dH, double* dE,
                            double* dG, hipStream_t st) {
  energy_any(L, prec, dL, dS, dH, dE, st);
  if (prec == LSDM_FP64) lnv_backward<double>(L, dG, st);
  else if (prec == LSDM_FP32) lnv_backward<float>(L, dG, st);
  else if (prec == LSDM_BF16) lnv_backward_bf16(L, dG, st);
  else lnv_backward_rc(L, dG, st);
}
static double read_scalar(const double* d, hipStream_t st) {
  double h = 0;
  HIP_CHECK(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  return h;
}

// coefficients c[0..3] of E(L + tD) from energies at t = -h, 0, h, 2h; Lt is
// an L-sized workspace, dE one device double
static void line_coeffs(lsdm_lnv* L, int prec, const double* dL, const double* dD, const double* dS, const double* dH,
                        double h, double* c, double* Lt, double* dE, hipStream_t st) {
  const i64 n = L->pL->nval;
  double e[4];
  const double ts[4] = {-1.0, 0.0, 1.0, 2.0};
  for (int k = 0; k < 4; ++k) {
    lincomb(Lt, dL, dD, 1.0, ts[k] * h, n, st);
    energy_any(L, prec, Lt, dS, dH, dE, st);
    check_launch();
    e[k] = read_scalar(dE, st);
  }
  // E(s h) = a0 + a1 s + a2 s^2 + a3 s^3 through s = -1, 0, 1, 2
  const double a0 = e[1];
  const double a2 = 0.5 * (e[2] + e[0]) - a0;
  const double odd = 0.5 * (e[2] - e[0]);                       // a1 + a3
  const double a3 = (0.5 * (e[3] - a0 - 4.0 * a2) - odd) / 3.0;  // (a1 + 4 a3 - (a1 + a3)) / 3
  const double a1 = odd - a3;
  c[0] = a0;
  c[1] = a1 / h;
  c[2] = a2 / (h * h);
  c[3] = a3 / (h * h * h);
}

// the same coefficients when c0 = E(L) and c1 = <dE/dL, D> are already known
// (inside the minimiser): energies at t = -h and h give the even and odd parts,
// so two chain evaluations instead of four and an exact slope
static void line_coeffs_known(lsdm_lnv* L, int prec, const double* dL, const double* dD, const double* dS,
                              const double* dH, double h, double c0, double c1, double* c, double* Lt, double* dE,
                              hipStream_t st) {
  const i64 n = L->pL->nval;
  double e[2];
  for (int k = 0; k < 2; ++k) {
    lincomb(Lt, dL, dD, 1.0, (k ? 1.0 : -1.0) * h, n, st);
    energy_any(L, prec, Lt, dS, dH, dE, st);
    check_launch();
    e[k] = read_scalar(dE, st);
  }
  c[0] = c0;
  c[1] = c1;
  c[2] = (0.5 * (e[1] + e[0]) - c0) / (h * h);          // c2 h^2
  c[3] = (0.5 * (e[1] - e[0]) - c1 * h) / (h * h * h);  // c1 h + c3 h^3
}

// step to the local minimum of c1 t + c2 t^2 + c3 t^3 along a descent
// direction (c1 < 0); fallback when the cubic has none: t = h
static double cubic_step(const double* c, double h) {
  const double c1 = c[1], c2 = c[2], c3 = c[3];
  const double disc = c2 * c2 - 3.0 * c1 * c3;
  double t = -1.0;
  if (disc >= 0.0) {
    const double den = c2 + std::sqrt(disc);   // the root where 2 c2 + 6 c3 t > 0
    if (den > 0.0) t = -c1 / den;
  }
  if (!(t > 0.0) || !std::isfinite(t)) t = h;
  return t;
}

int lsdm_lnv_line(lsdm_lnv* L, int prec, const double* dL, const double* dD, const double* dS, const double* dH,
                  double h, double* coeffs, void* stream) {
  return guarded([&] {
    require_device();
    if (!L || !dL || !dD || !dS || !dH || !coeffs) LSDM_THROW(LSDM_EINVAL, "null argument");
    if (!(h > 0.0) || !std::isfinite(h)) LSDM_THROW(LSDM_EINVAL, "h must be finite and > 0");
    hipStream_t st = (hipStream_t)stream;
    DevBuf Lt, dE;
    Lt.alloc(sizeof(double) * std::max<i64>(1, L->pL->nval));
    dE.alloc(sizeof(double));
    line_coeffs(L, prec, dL, dD, dS, dH, h, coeffs, Lt.as<double>(), dE.as<double>(), st);
  });
}

int lsdm_lnv_minimise(lsdm_lnv* L, int prec, double* dL, const double* dS, const double* dH, int max_iter,
                      double gtol, double h0, double* E_hist, double* gnorm_hist, int* iters, void* stream) {
  return guarded([&] {
    require_device();
    if (!L || !dL || !dS || !dH || !E_hist || !gnorm_hist || !iters) LSDM_THROW(LSDM_EINVAL, "null argument");
    if (max_iter < 0 || !(gtol >= 0.0) || !(h0 > 0.0) || !std::isfinite(h0))
      LSDM_THROW(LSDM_EINVAL, "max_iter >= 0, gtol >= 0 and a finite h0 > 0 are required");
    hipStream_t st = (hipStream_t)stream;
    const i64 n = L->pL->nval;
    const size_t nb = sizeof(double) * std::max<i64>(1, n);
    DevBuf G, Gn, D, Lt, sc, part;
    G.alloc(nb); Gn.alloc(nb); D.alloc(nb); Lt.alloc(nb);
    sc.alloc(sizeof(double) * 4);
    part.alloc(sizeof(double) * 2 * DOT_BLOCKS);
    double* dE = sc.as<double>();
    double* dd = sc.as<double>() + 1;
    auto dotp = [&](const double* a, const double* b) {
      dot(a, b, n, 1.0, part.as<double>(), dd, st);
      return read_scalar(dd, st);
    };
    energy_grad_any(L, prec, dL, dS, dH, dE, G.as<double>(), st);
    check_launch();
    E_hist[0] = read_scalar(dE, st);
    double g2 = dotp(G.as<double>(), G.as<double>());
    gnorm_hist[0] = std::sqrt(g2);
    lincomb(D.as<double>(), G.as<double>(), G.as<double>(), -1.0, 0.0, n, st);   // D = -G
    double h = h0;
    double slope = -g2;                                                          // <G, D>
    int it = 0;
    while (it < max_iter && std::sqrt(g2) > gtol) {
      double c[4];
      line_coeffs_known(L, prec, dL, D.as<double>(), dS, dH, h, E_hist[it], slope, c, Lt.as<double>(), dE, st);
      const double t = cubic_step(c, h);
      lincomb(dL, dL, D.as<double>(), 1.0, t, n, st);                            // L += t D
      energy_grad_any(L, prec, dL, dS, dH, dE, Gn.as<double>(), st);
      check_launch();
      ++it;
      E_hist[it] = read_scalar(dE, st);
      const double gn2 = dotp(Gn.as<double>(), Gn.as<double>());
      const double gng = dotp(Gn.as<double>(), G.as<double>());
      const double beta = std::max(0.0, (gn2 - gng) / g2);                       // Polak-Ribiere+
      lincomb(D.as<double>(), Gn.as<double>(), D.as<double>(), -1.0, beta, n, st);  // D = -Gn + beta D
      slope = dotp(D.as<double>(), Gn.as<double>());
      if (slope >= 0.0) {                                                        // not a descent direction
        lincomb(D.as<double>(), Gn.as<double>(), Gn.as<double>(), -1.0, 0.0, n, st);
        slope = -gn2;
      }
      G.swap(Gn);
      g2 = gn2;
      gnorm_hist[it] = std::sqrt(g2);
      h = t;
    }
    *iters = it;
    HIP_CHECK(hipStreamSynchronize(st));
  });
}

// ---------------------------------------------------------------------------
// Electron number (section 2, constraint 2: N_e = 2 Tr(KS)).  A chemical
// potential enters as H - mu S, so that 2 Tr[K(H - mu S)] = E - mu N_e and the
// same chain minimises the grand potential; N_e itself is the chain's energy
// with H replaced by S (S's range lies inside H's, and K lives on H's range).
// ---------------------------------------------------------------------------
static void s2h_map(lsdm_lnv* L) {
  std::lock_guard<std::mutex> g(L->s2h_mutex);
  if (L->s2h_ready) return;
  const lsdm_pattern *S = L->pS, *H = L->pH;
  const i64 nb = (i64)S->col.size();
  std::vector<i64> so(nb), ho(nb);
  std::vector<i32> sz(nb);
  for (i32 i = 0; i < L->sys->n_atoms; ++i) {
    for (i64 b = S->row_ptr[i]; b < S->row_ptr[i + 1]; ++b) {
      const i64 key = ((i64)S->col[b] << 24) | (i64)S->img[b];
      i64 lo = H->row_ptr[i], hi = H->row_ptr[i + 1];
      while (lo < hi) {                       // H's rows are sorted by (column, image)
        const i64 mid = (lo + hi) >> 1;
        if ((((i64)H->col[mid] << 24) | (i64)H->img[mid]) < key) lo = mid + 1; else hi = mid;
      }
      if (lo >= H->row_ptr[i + 1] || (((i64)H->col[lo] << 24) | (i64)H->img[lo]) != key)
        LSDM_THROW(LSDM_EPATTERN, "S's pattern is not contained in H's (rS > rH)");
      so[b] = S->val_off[b];
      ho[b] = H->val_off[lo];
      sz[b] = L->sys->nfn[i] * L->sys->nfn[S->col[b]];
    }
  }
  L->d_s2h_s.upload(so.data(), sizeof(i64) * nb);
  L->d_s2h_h.upload(ho.data(), sizeof(i64) * nb);
  L->d_s2h_n.upload(sz.data(), sizeof(i32) * nb);
  L->n_sblk = nb;
  L->s2h_ready = true;
}

// out = beta H + alpha S on H's pattern (dH may be null when beta = 0)
static void shift_into(lsdm_lnv* L, double alpha, const double* dS, double beta, const double* dH, double* dOut,
                       hipStream_t st) {
  s2h_map(L);
  const i64 n = L->pH->nval;
  if (dH) lincomb(dOut, dH, dH, beta, 0.0, n, st);
  else fill<double>(dOut, n, 0.0, st);
  add_blocks(dOut, dS, L->d_s2h_s.as<i64>(), L->d_s2h_h.as<i64>(), L->d_s2h_n.as<i32>(), L->n_sblk, alpha, st);
  check_launch();
}

int lsdm_lnv_shift(lsdm_lnv* L, double alpha, const double* dS, double beta, const double* dH, double* dOut,
                   void* stream) {
  return guarded([&] {
    require_device();
    if (!L || !dS || !dOut || (!dH && beta != 0.0)) LSDM_THROW(LSDM_EINVAL, "null argument");
    if (!std::isfinite(alpha) || !std::isfinite(beta)) LSDM_THROW(LSDM_EINVAL, "alpha and beta must be finite");
    shift_into(L, alpha, dS, beta, dH, dOut, (hipStream_t)stream);
  });
}

int lsdm_lnv_electrons(lsdm_lnv* L, int prec, const double* dL, const double* dS, double* dN, double* dGradN,
                       void* stream) {
  return guarded([&] {
    require_device();
    if (!L || !dL || !dS || !dN) LSDM_THROW(LSDM_EINVAL, "null argument");
    if (prec < LSDM_FP64 || prec > LSDM_FP32_RC) LSDM_THROW(LSDM_EINVAL, "unknown precision mode");
    hipStream_t st = (hipStream_t)stream;
    {
      std::lock_guard<std::mutex> g(L->s2h_mutex);
      if (!L->wSh.p) L->wSh.alloc(sizeof(double) * std::max<i64>(1, L->pH->nval));
    }
    shift_into(L, 1.0, dS, 0.0, nullptr, L->wSh.as<double>(), st);
    if (dGradN) energy_grad_any(L, prec, dL, dS, L->wSh.as<double>(), dN, dGradN, st);
    else energy_any(L, prec, dL, dS, L->wSh.as<double>(), dN, st);
    check_launch();
  });
}

int lsdm_lnv_purify(lsdm_lnv* L, int prec, const double* dL, const double* dS, double* dLout, void* stream) {
  return guarded([&] {
    require_device();
    if (!L || !dL || !dS || !dLout) LSDM_THROW(LSDM_EINVAL, "null argument");
    if (dLout == dL) LSDM_THROW(LSDM_EINVAL, "dLout must not alias dL");
    purify_build(L);
    hipStream_t st = (hipStream_t)stream;
    if (prec == LSDM_FP64) purify_chain<double>(L, dL, dS, dLout, st);
    else if (prec == LSDM_FP32) purify_chain<float>(L, dL, dS, dLout, st);
    else if (prec == LSDM_BF16 || prec == LSDM_FP32_RC) LSDM_THROW(LSDM_EUNSUPPORTED, "purification runs in FP64 or FP32");
    else LSDM_THROW(LSDM_EINVAL, "unknown precision mode");
  });
}

int lsdm_lnv_energy(lsdm_lnv* L, int prec, const double* dL, const double* dS, const double* dH, double* dK,
                    double* dE, void* stream) {
  return guarded([&] {
    require_device();
    if (!L || !dL || !dS || !dH || !dE) LSDM_THROW(LSDM_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    if (prec == LSDM_FP64) lnv_forward<double>(L, dL, dS, dH, dK, dE, st);
    else if (prec == LSDM_FP32) lnv_forward<float>(L, dL, dS, dH, dK, dE, st);
    else if (prec == LSDM_BF16) lnv_forward_bf16(L, dL, dS, dH, dK, dE, st);
    else if (prec == LSDM_FP32_RC) lnv_forward_rc(L, dL, dS, dH, dK, dE, st);
    else LSDM_THROW(LSDM_EINVAL, "unknown precision mode");
  });
}

int lsdm_lnv_energy_grad(lsdm_lnv* L, int prec, const double* dL, const double* dS, const double* dH, double* dE,
                         double* dG, void* stream) {
  return guarded([&] {
    require_device();
    if (!L || !dL || !dS || !dH || !dE || !dG) LSDM_THROW(LSDM_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    if (prec == LSDM_FP64) {
      // symmetric mode: E without P (the same value; see lnv_forward)
      lnv_forward<double>(L, dL, dS, dH, nullptr, dE, st, L->sym);
      lnv_backward<double>(L, dG, st, L->sym ? dE : nullptr);
    } else if (prec == LSDM_FP32) {
      lnv_forward<float>(L, dL, dS, dH, nullptr, dE, st);
      lnv_backward<float>(L, dG, st);
    } else if (prec == LSDM_BF16) {
      lnv_forward_bf16(L, dL, dS, dH, nullptr, dE, st);
      lnv_backward_bf16(L, dG, st);
    } else if (prec == LSDM_FP32_RC) {
      lnv_forward_rc(L, dL, dS, dH, nullptr, dE, st);
      lnv_backward_rc(L, dG, st);
    } else {
      LSDM_THROW(LSDM_EINVAL, "unknown precision mode");
    }
  });
}

int lsdm_lnv_profile(lsdm_lnv* L, int enable) {
  return guarded([&] {
    if (!L) LSDM_THROW(LSDM_EINVAL, "null argument");
    L->prof = enable != 0;
    L->ev_used = 0;
    L->ev_prod.clear();
  });
}

int lsdm_lnv_profile_read(lsdm_lnv* L, double* ms, int64_t* launches, double* flops) {
  return guarded([&] {
    if (!L || !ms || !launches || !flops) LSDM_THROW(LSDM_EINVAL, "null argument");
    for (int w = 0; w < 8; ++w) {
      ms[w] = 0.0;
      launches[w] = 0;
      flops[w] = chain_plan(L, w) ? chain_plan(L, w)->flops : 0.0;   // symmetric mode has no B4 product
    }
    if (L->ev_used) HIP_CHECK(hipEventSynchronize(L->ev_pool[L->ev_used - 1]));
    for (size_t k = 0; k < L->ev_prod.size(); ++k) {
      float t = 0.f;
      HIP_CHECK(hipEventElapsedTime(&t, L->ev_pool[2 * k], L->ev_pool[2 * k + 1]));
      ms[L->ev_prod[k]] += t;
      launches[L->ev_prod[k]] += 1;
    }
    L->ev_used = 0;
    L->ev_prod.clear();
  });
}

void lsdm_lnv_destroy(lsdm_lnv* L) {
  if (!L) return;
  for (lsdm_plan* p : {L->F1, L->F2, L->F3, L->B1, L->B2, L->B3, L->B4, L->B5, L->P2, L->P3}) delete p;
  for (lsdm_pattern* p : {L->pS, L->pH, L->pL, L->pX, L->pM, L->pM2}) delete p;
  delete L;
}

}  // extern "C"
