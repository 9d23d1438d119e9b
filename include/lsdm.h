/*
 * lsdm.h - C ABI of the MI355X (gfx950) library for the hot path of the LNV
 * linear-scaling density-matrix method: atom-blocked sparse products truncated
 * to spherical interatomic ranges, the McWeeny/LNV density matrix
 * K = 3LSL - 2LSLSL, the energy E = 2 Tr(KH) and its gradient dE/dL.
 *
 * Source of the operations: Bowler & Miyazaki, "Calculations on millions of
 * atoms with DFT: linear scaling shows its potential", section 2 (Methodology):
 *   - eq. 1 and eq. 2 index matrices by (atom, support function), so every
 *     matrix here is a set of dense atom blocks of size nfn_i x nfn_j;
 *   - the range cutoff on L stated after eq. 3 (an element is zero when the
 *     interatomic distance exceeds the range) defines a range pattern;
 *   - item 1 of the list of computational operations is the sparse matrix
 *     multiplication (the example K_ij = L_ik S_kl L_lj);
 *   - eq. 3 defines K from L and S; the electron-count constraint
 *     N_e = 2 Tr(KS) fixes the spin factor 2 used in E = 2 Tr(KH).
 *
 * Conventions shared by every call
 *   Units: positions and ranges in bohr (any consistent length unit works).
 *   Periodicity: `lattice` holds three row vectors (9 doubles, row-major) or is
 *     NULL for an open system.  Periodic matrices are image-resolved: a block
 *     is keyed (i, j, n), n an integer translation applied to atom j, so ranges
 *     larger than half the cell are exact (no folding).
 *   Range test: a pair is in a pattern of range R iff
 *     |x_j + n.T - x_i|^2 <= R^2 in IEEE double (a pair exactly at R is kept).
 *   Value layout ("block layout"): the blocks of a pattern in row order, each
 *     row sorted by (j, n0, n1, n2); block b is nfn_i x nfn_j row-major and
 *     starts at val_off[b] (exported by lsdm_pattern_export).  Value arrays
 *     passed to the library are DEVICE pointers to doubles in this layout.
 *   Ownership: handles are created and destroyed by the library; value
 *     buffers belong to the caller and are never freed by the library.  Device
 *     workspace is allocated by the library (hipMalloc, or the caller's
 *     allocator: lsdm_set_allocator) when a handle is
 *     created or first used and released when it is destroyed: a plan keeps
 *     the operand workspaces of its stand-alone multiplies and the two plans
 *     of its adjoint, so repeated calls on one plan allocate nothing.
 *   Streams: compute calls enqueue work on `stream` (a hipStream_t, NULL = the
 *     default stream).  The multiplies, the dots and the LNV energy,
 *     gradient, shift and electron calls return without waiting; *_create
 *     calls, the line search and the minimiser (which read scalars back)
 *     synchronise, and so does the first call that builds a lazy
 *     part of a handle (layout maps, adjoint plans, residual-mode maps, the
 *     S-in-H map, the dot's partial sums).  Calls on one handle must not run
 *     concurrently, on one stream or several: they share the handle's
 *     workspaces (calls queued one after another on one stream are fine).
 *   Errors: every call returns LSDM_OK (0) or a negative status; no exception
 *     crosses the ABI; lsdm_last_error() returns a message for the calling
 *     thread's last failure.  A failed call leaves its outputs undefined and
 *     its handles valid.
 */
#ifndef LSDM_H
#define LSDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsdm_system lsdm_system;
typedef struct lsdm_pattern lsdm_pattern;
typedef struct lsdm_plan lsdm_plan;
typedef struct lsdm_lnv lsdm_lnv;

enum {
  LSDM_OK = 0,
  LSDM_EINVAL = -1,        /* bad argument (NULL, NaN position, range < 0, nfn out of 1..16, ...) */
  LSDM_EPATTERN = -2,      /* patterns of different systems combined */
  LSDM_ENOMEM = -3,        /* device or host allocation failed, or a size limit was exceeded */
  LSDM_EDEVICE = -4,       /* a HIP call failed */
  LSDM_EUNSUPPORTED = -5   /* valid request the library does not implement */
};

/* Precision of the block products.  Traces, energies and K assembly are FP64
 * in every mode. */
enum {
  LSDM_FP64 = 0,    /* FP64 inputs, FP64 MFMA, FP64 accumulation */
  LSDM_FP32 = 1,    /* inputs rounded to FP32, FP32 MFMA, FP32 accumulation */
  LSDM_BF16 = 2,    /* inputs rounded to BF16, BF16 MFMA, FP32 accumulation */
  LSDM_FP32_RC = 3  /* FP32 products of the off-site parts plus FP64 on-site
                       (block-diagonal) terms, see lsdm_multiply */
};

/* ---- device memory ----------------------------------------------------- */
/* Allocator of the library's internal device workspaces (value buffers stay
 * the caller's).  With alloc and release both non-NULL, every later workspace
 * allocation calls alloc(bytes, ctx), which must return memory of the
 * current HIP device, at least `bytes` long and aligned to 256 bytes, or
 * NULL: the library call that asked then fails with LSDM_ENOMEM (and with
 * LSDM_EINVAL for a misaligned pointer, which it gives back at once).  A
 * workspace goes back through release(ptr, ctx) of the allocator that made
 * it, when its handle is destroyed or the workspace is resized.  Both NULL
 * restores hipMalloc / hipFree.  The setting is process-wide.  Buffers made
 * before a change keep the allocator that made them, so a pair must stay
 * callable until every handle that used it is destroyed.  Both functions are
 * called on the thread that calls the library, never from device code or
 * a stream callback.  A workspace is used on the streams of the calls that
 * use it, so a stream-ordered allocator must not hand released memory out
 * again before that work is complete.
 * Errors: LSDM_EINVAL (exactly one of alloc and release NULL). */
typedef void* (*lsdm_alloc_fn)(size_t bytes, void* ctx);
typedef void (*lsdm_free_fn)(void* ptr, void* ctx);
int lsdm_set_allocator(lsdm_alloc_fn alloc, lsdm_free_fn release, void* ctx);

/* ---- system ------------------------------------------------------------ */
/* Atoms with orbital blocks (eq. 1: support functions i-alpha on atom i).
 * xyz: host, 3*n_atoms doubles.  nfn: host, n_atoms values in 1..16.
 * lattice: host, 9 doubles (rows are the translation vectors) or NULL.
 * Positions must be finite; periodic positions may lie outside the cell.
 * Errors: LSDM_EINVAL (n_atoms < 1, a null pointer, a non-finite position,
 * nfn outside 1..16, a singular lattice). */
int lsdm_system_create(int32_t n_atoms, const double* xyz, const int32_t* nfn,
                       const double* lattice, lsdm_system** out);
void lsdm_system_destroy(lsdm_system* sys);

/* ---- range patterns (symbolic pass, step 1) ----------------------------- */
/* Pattern of all blocks (i, j, n) within `range` (the locality cutoff stated
 * after eq. 3), found by a cell-list neighbour search (on the device when
 * there is one, one thread per atom, rows key-sorted; on the host otherwise),
 * then laid out in the internal strip layout on the device.
 * Errors: LSDM_EINVAL (range < 0 or not finite), LSDM_ENOMEM (the pattern
 * would exceed the device or an index limit), LSDM_EDEVICE. */
int lsdm_pattern_create(const lsdm_system* sys, double range, lsdm_pattern** out);
/* Number of blocks and of values (doubles) of the block layout. */
int lsdm_pattern_info(const lsdm_pattern* p, int64_t* n_blocks, int64_t* n_values);
/* Copy the pattern to HOST arrays: row_ptr[n_atoms+1], col[n_blocks],
 * img3[3*n_blocks] (the image n of each block, components in -127..127),
 * val_off[n_blocks].  Any output pointer may be NULL. */
int lsdm_pattern_export(const lsdm_pattern* p, int64_t* row_ptr, int32_t* col,
                        int8_t* img3, int64_t* val_off);
void lsdm_pattern_destroy(lsdm_pattern* p);

/* ---- truncated products (symbolic pass step 2 and the product) ---------- */
/* Plan for C = P_C(op(A) op(B)): the exact product of op(A) and op(B)
 * projected on C's pattern (C's range is the truncation), op = transpose when
 * the flag is 1.  A transposed operand uses A's pattern mirrored
 * ((i,j,n) -> (j,i,-n)).  The plan holds the task list of block triples
 * (i,k,j) grouped into tiles (16 output rows x 32 output columns of pseudo-
 * atoms) and steps (one inner pseudo-atom k of a tile) for the GPU kernels:
 * the tiles and their inner lists are built on the host (multithreaded), the
 * steps are generated and kept on the device.  The plan also holds the
 * per-XCD tile counters its product launches use, so one plan serves one
 * product at a time.  Without a device only the counts are computed
 * (plan_info works, products fail with LSDM_EDEVICE).
 * Errors: LSDM_EPATTERN (patterns of different systems), LSDM_ENOMEM. */
int lsdm_plan_create(const lsdm_pattern* A, int transA, const lsdm_pattern* B, int transB,
                     const lsdm_pattern* C, lsdm_plan** out);
/* n_triples: block triples (i,k,j) with (i,k) in op(A), (k,j) in op(B) and
 * (i,j) in C (the useful work); flops: sum over triples of 2 nfn_i nfn_k nfn_j;
 * plan_bytes: device memory held by the plan. */
int lsdm_plan_info(const lsdm_plan* plan, int64_t* n_triples, double* flops, int64_t* plan_bytes);
void lsdm_plan_destroy(lsdm_plan* plan);

/* C = alpha P_C(op(A) op(B)) + beta C, values in block layout on device.
 * dA, dB, dC: device doubles on the patterns given to lsdm_plan_create.
 * Asynchronous on the stream; the plan keeps the strip-layout copies of the
 * operands it needs (allocated on the first call in a precision), so calls
 * on one plan must be ordered (one stream, or synchronised between them).
 * prec: LSDM_FP64, LSDM_FP32, LSDM_BF16 or LSDM_FP32_RC.  In FP32_RC mode each
 * operand is split into its on-site blocks D (i = j, n = 0) and the rest R, and
 * AB = D_A B + A D_B - D_A D_B (FP64, block-diagonal scalings) + R_A R_B (FP32).
 * dC must not alias dA or dB.  Errors: LSDM_EINVAL, LSDM_EDEVICE. */
int lsdm_multiply(const lsdm_plan* plan, int prec, double alpha, const double* dA, const double* dB,
                  double beta, double* dC, void* stream);

/* Adjoint of the truncated product (the derivative of the multiply above):
 * for C = P_C(op(A) op(B)) and an upstream gradient dCbar on C's pattern,
 *   dAbar += P_A(Cbar op(B)^T)   (P_A(op(B) Cbar^T) when A enters transposed)
 *   dBbar += P_B(op(A)^T Cbar)   (P_B(Cbar^T op(A)) when B enters transposed)
 * Either output may be NULL (not computed).  Both accumulate.  Every
 * precision mode.  The two products' plans are built on the first call that
 * needs them (synchronous) and kept by the plan; later calls are
 * asynchronous.  Errors: LSDM_EINVAL, LSDM_ENOMEM, LSDM_EDEVICE. */
int lsdm_multiply_adjoint(const lsdm_plan* plan, int prec, const double* dCbar, const double* dA,
                          const double* dB, double* dAbar, double* dBbar, void* stream);

/* *dOut = sum over the blocks of p of <A_b, B_b>_F (= Tr(A B^T) over the
 * pattern; Tr(AB) for symmetric B).  FP64 with per-thread compensated sums and
 * a fixed-order tree, so the result is bitwise reproducible.  dOut: device.
 * Returns without waiting; its partial sums live on the pattern (16 KiB,
 * allocated on the first call), so later calls allocate nothing.
 * Errors: LSDM_EINVAL (null argument), LSDM_ENOMEM, LSDM_EDEVICE. */
int lsdm_dot(const lsdm_pattern* p, const double* dA, const double* dB, double* dOut, void* stream);
/* lsdm_dot without allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and the same result bit for bit; it allocates
 * nothing and does not synchronise (the result is ready when the stream
 * reaches it).  Its partial sums live in a static device array of the library
 * (16 KiB per device, held until the process ends; any pattern fits it, the
 * grid is fixed).  That array is shared by every call on a device: calls that
 * overlap on one device, on one stream or several, race.
 * Errors: LSDM_EINVAL (null argument), LSDM_EDEVICE. */
int lsdm_dot_noalloc(const lsdm_pattern* p, const double* dA, const double* dB, double* dOut, void* stream);

/* ---- the LNV chain ------------------------------------------------------- */
/* Patterns of S (range rS), H (rH) and L (rL) plus the intermediates
 * X = LS (the blocks that L S reaches, all within rL + rS), M = LSL
 * (min(2 rL + rS, rH + rL + rS)) and every plan of
 * the forward and adjoint chains.  These ranges drop only elements that cannot
 * reach K on H's range or dE/dL on L's range, so E and dE/dL equal the
 * untruncated algebra restricted to the S, H and L patterns.  Any ranges are
 * accepted; where rH > 2 rL + rS, LSL is zero on the blocks of H beyond its
 * range and K = -2 LSLSL there.
 * Errors: LSDM_EINVAL (a range < 0), LSDM_ENOMEM, LSDM_EDEVICE. */
int lsdm_lnv_create(const lsdm_system* sys, double rS, double rH, double rL, lsdm_lnv** out);
/* Flags of lsdm_lnv_create_ex. */
enum {
  /* Symmetric inputs (section 2: S and H of a real basis, and L built like K,
   * are symmetric: block (j,i,-n) = block (i,j,n)^T).  M = LSL, P = LSLSL and
   * dE/dL are then symmetric too.  The products X L and X M compute one half
   * of their output strips; the other half is the transpose of the first
   * (X L's epilogue writes it, the other consumers read the mirror blocks), and
   * the adjoint takes dE/dL as V + V^T - 4 X^T H X with X = LS and
   * V = 6 HX - 4 HMS (the same terms as the gradient of eq. 3, regrouped;
   * HX formed once on M's range and reused for both terms, X^T H X on one
   * half).  Every L passed to a handle made with this flag
   * (also L + tD in a line search) must be symmetric; for a non-symmetric L
   * the results are those of the computed half mirrored, not of eq. 3. */
  LSDM_LNV_SYMMETRIC = 1
};
/* lsdm_lnv_create with flags (0 or LSDM_LNV_SYMMETRIC).
 * Errors: as lsdm_lnv_create, and LSDM_EINVAL for an unknown flag. */
int lsdm_lnv_create_ex(const lsdm_system* sys, double rS, double rH, double rL, int flags, lsdm_lnv** out);
/* Borrowed views of the chain's patterns (owned by the lnv handle):
 * which = 0 S, 1 H, 2 L, 3 X, 4 M. */
int lsdm_lnv_pattern(const lsdm_lnv* lnv, int which, const lsdm_pattern** out);
/* Work of one energy (grad = 0) or energy+gradient (grad = 1) evaluation:
 * useful block triples and flops summed over the chain's products. */
int lsdm_lnv_info(const lsdm_lnv* lnv, int grad, int64_t* n_triples, double* flops);
/* K = 3 LSL - 2 LSLSL on H's pattern (eq. 3) and E = 2 <K, H> (FP64).
 * dL, dS, dH: device doubles in block layout on the L, S, H patterns (symmetric
 * matrices: block (j,i,-n) is the transpose of block (i,j,n)).
 * dK: device, H's pattern, may be NULL.  dE: device, one double. */
int lsdm_lnv_energy(lsdm_lnv* lnv, int prec, const double* dL, const double* dS, const double* dH,
                    double* dK, double* dE, void* stream);
/* E as above and dGradL = dE/dL on L's pattern, the derivative of eq. 3 with
 * respect to each stored entry of L (blocks (i,j,n) and (j,i,-n) independent):
 *   6 (HLS + SLH) - 4 (HLSLS + SLHLS + SLSLH)
 * computed by the adjoint chain of the truncated products, in the same
 * precision mode as the forward products.  dGradL: device.  In symmetric
 * mode at FP64 the energy skips P: Tr(PH) = <X, HM> for symmetric M and H,
 * and the adjoint forms -4 HM on X's pattern anyway, so E = 2 <3 M|_H, H> +
 * <X, -4 HM>; the value equals that of lsdm_lnv_energy up to rounding (not
 * bit for bit) and the call runs one product fewer. */
int lsdm_lnv_energy_grad(lsdm_lnv* lnv, int prec, const double* dL, const double* dS, const double* dH,
                         double* dE, double* dGradL, void* stream);
/* Exact line search (section 2: the ground state is the minimum of E over L;
 * eq. 3 makes E a cubic polynomial of L).  coeffs[0..3] (host) receive c0..c3
 * of E(L + tD) = c0 + c1 t + c2 t^2 + c3 t^3, obtained from the energies at
 * t = -h, 0, h, 2h (exact for a cubic up to rounding; choose h near the
 * expected step).  dL, dD: device, L's pattern.  Synchronises the stream.
 * Errors: LSDM_EINVAL (null pointer, h not finite or <= 0), LSDM_EDEVICE. */
int lsdm_lnv_line(lsdm_lnv* lnv, int prec, const double* dL, const double* dD, const double* dS, const double* dH,
                  double h, double* coeffs, void* stream);
/* Minimise E over L (in place, device, L's pattern) by Polak-Ribiere
 * conjugate gradients (beta clipped at 0, restart when the direction is not a
 * descent direction) with the exact line search above: each step goes to the
 * local minimum of the cubic along the direction (h = h0 for the first line,
 * then the previous step; if the cubic has no local minimum the step is h).
 * Inside the loop c0 and c1 = <dE/dL, D> are known, so each line costs two
 * chain evaluations (t = -h, h) on top of one energy-and-gradient pass.
 * Stops after max_iter steps or when |dE/dL| <= gtol (Frobenius norm over L's
 * stored values).  Host outputs: E_hist[0..iters] and gnorm_hist[0..iters]
 * (sized max_iter + 1), iters.  Scalars are read back every step.
 * Errors: LSDM_EINVAL, LSDM_ENOMEM, LSDM_EDEVICE. */
int lsdm_lnv_minimise(lsdm_lnv* lnv, int prec, double* dL, const double* dS, const double* dH, int max_iter,
                      double gtol, double h0, double* E_hist, double* gnorm_hist, int* iters, void* stream);
/* Chemical potential (section 2, constraint 2 on the electron number): with
 * H' = H - mu S the chain's energy is 2 Tr[K(H - mu S)] = E - mu N_e, so the
 * calls above evaluate and minimise the grand potential at fixed mu.
 * dOut = beta dH + alpha dS on H's pattern (device, H's value layout; S's
 * blocks are added at their place in H).  dH may be NULL when beta = 0 and may
 * equal dOut.  Asynchronous on the stream; the first call on a handle builds a
 * block map (synchronous).  Errors: LSDM_EINVAL, LSDM_EPATTERN (rS > rH: S's
 * pattern is not inside H's), LSDM_EDEVICE. */
int lsdm_lnv_shift(lsdm_lnv* lnv, double alpha, const double* dS, double beta, const double* dH, double* dOut,
                   void* stream);
/* Electron number N_e = 2 Tr(KS) with K of eq. 3 on H's range (section 2,
 * constraint 2), written to dN (device, one double), and optionally
 * dGradN = dN_e/dL on L's pattern (device, NULL to skip), in precision mode
 * prec.  Uses a workspace of H's size held by the handle; calls on one handle
 * must not overlap.  Errors: LSDM_EINVAL, LSDM_EPATTERN (rS > rH), LSDM_ENOMEM,
 * LSDM_EDEVICE. */
int lsdm_lnv_electrons(lsdm_lnv* lnv, int prec, const double* dL, const double* dS, double* dN, double* dGradN,
                       void* stream);
/* One McWeeny purification step (section 2: eq. 3 read as a map of L, whose
 * fixed points are idempotent LS): dLout = P_L(3 LSL - 2 LSLSL), both on L's
 * pattern (device), with every intermediate on the range it needs for an
 * exact result on L's range (LSL on 2 rL + rS).  The first call builds that
 * pattern and two plans (synchronous).  Track the electron number of the
 * iterates with lsdm_lnv_electrons.  prec: LSDM_FP64 or LSDM_FP32.
 * dLout must not alias dL.  Errors: LSDM_EINVAL, LSDM_EUNSUPPORTED (BF16 or
 * FP32_RC), LSDM_ENOMEM, LSDM_EDEVICE. */
int lsdm_lnv_purify(lsdm_lnv* lnv, int prec, const double* dL, const double* dS, double* dLout, void* stream);
/* Kernel timing of the chain's products: with enable = 1 every product launch
 * of lsdm_lnv_energy(_grad) is bracketed by HIP events recorded on the call's
 * stream (no extra synchronisation); enable = 0 stops and discards. */
int lsdm_lnv_profile(lsdm_lnv* lnv, int enable);
/* Waits for the recorded events, then returns per product (F1 F2 F3 B1 B2 B3
 * B4 B5; host arrays of 8) the summed kernel milliseconds, the number of
 * launches and the useful flops of one launch; clears the record.  F1-F3 make
 * X = LS, M = XL and P = XM; B1 Mbar = X^T Pbar, B2 Xbar = Pbar M, then
 * B3 Xbar += Mbar L, B4 dE/dL = X^T Mbar, B5 dE/dL += Xbar S, or in symmetric
 * mode B1 Y = HX, B3 dE/dL = -4 X^T Y, B5 V = Xbar S + 6 Y on L's range (B4
 * has no launches and no flops) and dE/dL += V + V^T; a symmetric FP64
 * energy-and-gradient call launches no F3 (its energy skips P). */
int lsdm_lnv_profile_read(lsdm_lnv* lnv, double* ms, int64_t* launches, double* flops);
void lsdm_lnv_destroy(lsdm_lnv* lnv);

/* Message of the calling thread's last failed call ("" if none). */
const char* lsdm_last_error(void);
/* Library version string. */
const char* lsdm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LSDM_H */
