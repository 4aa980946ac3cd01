/*
 * gpuqt.h -- C ABI of the MI355X (gfx950) Chebyshev / KPM linear-scaling Kubo
 * transport library.
 *
 * Method: Fan, Vierimaa & Harju, "GPUQT: an efficient linear-scaling quantum
 * transport code fully implemented on graphics processing units"
 * (Comput. Phys. Commun.; arXiv:1705.01387).  hbar = 1 (Section 4.2.6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Complex numbers are interleaved {double re, double im} (the memory layout
 *    of torch.complex128 / C99 double complex).  A "c128 pointer" below is a
 *    `double*` to such pairs and must be 16-byte aligned.
 *  - State vectors hold B columns in layout [n][B] (column index fastest):
 *    element (i, b) is at c128 offset i*B + b.  B is 1, 2, 4, 8 or 16.
 *  - Unless stated otherwise, vector, output and workspace pointers are DEVICE
 *    pointers owned by the caller; the library never frees them.  Descriptor
 *    arrays passed to gpuqt_build_h and the `dt` arrays of gpuqt_vac/gpuqt_msd
 *    are HOST pointers, read during the call only.
 *  - Compute calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*; NULL = the null stream).  All argument checks happen on the host
 *    before anything is enqueued; a call that returns an error has enqueued
 *    nothing.  Results are valid once the stream has reached the call.
 *  - Compute calls never allocate device memory: scratch comes from the
 *    caller's workspace, sized by gpuqt_workspace_size.  Two calls that run at
 *    the same time on one handle need distinct workspaces.
 *  - No entry point throws or aborts.  Each returns a gpuqt_status; on failure
 *    gpuqt_last_error() gives a message (per thread).
 */
#ifndef GPUQT_H
#define GPUQT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gpuqt_status;
enum {
  GPUQT_OK = 0,
  GPUQT_ERR_ARG = 1,         /* null pointer, size out of range, misaligned or aliased buffer */
  GPUQT_ERR_LAYOUT = 2,      /* neighbour index out of range, count > max_nn, bond between
                                segments, non-Hermitian H, bond of exactly half the period */
  GPUQT_ERR_SPECTRUM = 3,    /* DeltaE below the Gershgorin bound, or |E| >= DeltaE */
  GPUQT_ERR_WORKSPACE = 4,   /* workspace smaller than gpuqt_workspace_size */
  GPUQT_ERR_HIP = 5,         /* HIP runtime failure (no device, launch error, wrong device) */
  GPUQT_ERR_NOMEM = 6,       /* device allocation failed (gpuqt_build_h only) */
  GPUQT_ERR_UNSUPPORTED = 7  /* valid request this build does not handle (e.g. B = 3) */
};

typedef struct gpuqt_h_s *gpuqt_h;   /* opaque handle of a Hamiltonian on one device */

/*
 * Tight-binding model, as the paper's input files describe it (Section 4.2):
 *   H = sum_mn H_mn |m><n| + sum_m U_m |m><m|,  X = diag(x),
 *   V = i [H, X],  (V)_mn = i (x_n - x_m) H_mn.
 * Several independent systems ("segments": disorder realisations of any
 * sizes) may be stacked block-diagonally; each gets its own DeltaE, and every
 * moment is then reported per segment.
 */
typedef struct {
  int64_t n;                    /* number of orbitals (all segments), >= 1 */
  int32_t max_nn;               /* neighbour slots per orbital (Section 4.2.1), >= 0 */
  const int32_t *nn;            /* [n] neighbour count of each orbital, 0..max_nn */
  const int32_t *nbr;           /* [n*max_nn] row-major: nbr[i*max_nn + s], s < nn[i], in [0, n) */
  const double *hop;            /* NULL: every hopping is -1 (Section 4.2.2);
                                   else [n*max_nn] real, or [2*n*max_nn] interleaved complex,
                                   hop[i*max_nn + s] = H[i, nbr[i*max_nn + s]] */
  int32_t hop_is_complex;       /* 0: real hoppings; 1: complex */
  const int32_t *hop_class;     /* NULL or [n*max_nn]: class of each hopping, for gradients */
  int32_t n_class;              /* number of hopping classes (>= 1) */
  const double *onsite;         /* NULL: U = 0 (Section 4.2.3); else [n] */
  const double *x;              /* [n] coordinate along the transport direction (Section 4.2.4) */
  double length_x;              /* period along x (minimum-image differences); <= 0: open */
  double volume;                /* system volume Omega (reported back; used by the caller) */
  double energy_max;            /* DeltaE (Section 3.2); <= 0: 1.01 x Gershgorin bound */
  int32_t n_segments;           /* 0 or 1: one system; > 1: block-diagonal segments */
  const int64_t *seg_offsets;   /* [n_segments+1] first row of each segment, last = n */
  const double *seg_energy_max; /* NULL or [n_segments]: per-segment DeltaE (<= 0: auto) */
  const double *seg_length_x;   /* NULL or [n_segments]: per-segment period (else length_x) */
  int32_t check_hermitian;      /* nonzero: require H_ji = conj(H_ij) (sums over duplicates) */
  int32_t slice_height;         /* sliced-ELL slice height: 0 = default (64), else 32..1024, 2^k */
  int32_t band_rows;            /* rows per band of the banded row order (see gpuqt_autotune):
                                   0 = chosen per block width (and, for B >= 2, two bands per
                                   period for periods of 1024 rows or more that fit in one
                                   band); else a
                                   multiple of 64, used for every width and every segment whose
                                   row period exceeds it */
  int32_t no_dictionary;        /* nonzero: keep one hopping per entry.  Otherwise, with at
                                   most 4 hopping classes, when the (column offset, hopping,
                                   position difference, class) tuples take at most 65,535
                                   distinct values (a uniform field, a few bond types) each
                                   entry stores a 16-bit index into a table of them (hop_mode 3
                                   in gpuqt_h_info_t) */
} gpuqt_h_desc;

/*
 * Build the device layout of H (sliced ELL: neighbour indices, hoppings
 * scaled by 1/DeltaE, position differences, on-site terms; Section 4.2).
 * Validates the descriptor (GPUQT_ERR_LAYOUT / GPUQT_ERR_SPECTRUM before any
 * device work), then allocates device memory on the current device and copies
 * synchronously.  *out receives a handle owned by the caller (gpuqt_destroy_h).
 * A DeltaE below the segment's Gershgorin bound max_i(|U_i| + sum_j |H_ij|) is
 * rejected (GPUQT_ERR_SPECTRUM): the paper requires the spectrum of H/DeltaE
 * to lie in [-1, 1] (Section 3.2, Section 4.2.7).
 */
gpuqt_status gpuqt_build_h(const gpuqt_h_desc *desc, void *stream, gpuqt_h *out);

/* Free the handle and its device memory (NULL is ignored).  The caller must
 * make sure no enqueued work still uses it. */
void gpuqt_destroy_h(gpuqt_h h);

/*
 * Replace model values in place (training loops, finite differences); DeltaE and the
 * neighbour structure stay fixed.
 *   onsite      : DEVICE double [n] or NULL: new on-site energies U_i (Section 4.2.3).
 *   class_scale : HOST double [n_class] or NULL: every hopping of class c becomes
 *                 class_scale[c] times the hopping given to gpuqt_build_h (at most 8 classes).
 * Then recomputes the Gershgorin bound of every segment on the device and returns
 * GPUQT_ERR_SPECTRUM if it exceeds the segment's DeltaE (the new values are kept; update
 * again before computing).  Synchronises the stream; the first class update allocates a
 * device copy of the build-time hoppings.  Not safe while other calls on the handle run.
 */
gpuqt_status gpuqt_update_h_values(gpuqt_h h, const double *onsite, const double *class_scale,
                                   void *stream);

typedef struct {
  int64_t n;                 /* orbitals */
  int32_t n_segments;
  int32_t n_class;
  int32_t hop_mode;          /* 0: one value per segment, 1: real, 2: complex per entry, 3: table */          /* 0: uniform value per segment, 1: real, 2: complex */
  int32_t slice_height;
  int64_t n_slices;
  int64_t entries;           /* stored ELL entries (with padding) */
  int64_t nnz;               /* neighbour entries (without padding) */
  int32_t max_width;         /* widest slice */
  int32_t uniform_width;     /* width of every slice when equal and unpadded, else 0 */
  int32_t grid_blocks;       /* workgroups per sparse-step launch */
  int32_t kernel_variant;    /* bit 0: non-temporal streams, bit 1: banded row order, bits 2-5:
                                per-CU workgroup cap (see gpuqt_autotune) */
  size_t device_bytes;       /* device memory held by the handle */
  int64_t row_period;        /* largest detected row period D over the segments (0: none) */
  int32_t banded_mask;       /* bit log2(B) set: block width B has a banded row order */
  int32_t family_caps;       /* per kernel family f (GPUQT_K_*), bits 4f..4f+3: 0 = the per-CU
                                cap of kernel_variant, else 1 + that family's own cap (1: none) */
  int32_t max_nn;            /* neighbour slots per row of the build descriptor: the row stride
                                of per-entry hopping gradients */
  int32_t pencil_mask;       /* bit log2(B) set: block width B has a pencil row order */
  int32_t box[3];            /* (Lx, Ly, Lz) when H is a periodic simple cubic box in natural
                                order with one uniform hopping (see gpuqt_autotune, bit 26),
                                else 0 */
  int32_t box_msd;           /* 1: on that box the position differences are +-dx for the x
                                neighbours and 0 for the others, so the MSD term can run as a
                                box stencil too (bit 27) */
  int32_t sheets;            /* 1: every segment is a periodic Lx x Ly square in natural order
                                (rows off_s + x + Lx y, each with its four periodic neighbours,
                                Lx, Ly >= 3, Lx Ly <= 2^24) with one uniform hopping, so the
                                Hermitian step can run as a sheet stencil (bit 26) */
} gpuqt_h_info_t;

/* Describe the layout.  energy_max (may be NULL) receives [n_segments] DeltaE;
 * gershgorin (may be NULL) the [n_segments] bounds. */
gpuqt_status gpuqt_h_info(gpuqt_h h, gpuqt_h_info_t *info, double *energy_max, double *gershgorin);

/* Operations, for gpuqt_workspace_size. */
enum {
  GPUQT_OP_MOMENTS = 0,
  GPUQT_OP_EVOLVE = 1,
  GPUQT_OP_EVOLVE_COMMUTATOR = 2,
  GPUQT_OP_VAC = 3,
  GPUQT_OP_MSD = 4,
  GPUQT_OP_MOMENTS_BACKWARD = 5,
  GPUQT_OP_AUTOTUNE = 6
};

/* Bytes of device workspace `op` needs for B columns, M moments and Np
 * Chebyshev terms per time step.  Np = 0 reserves room for up to 8192 terms
 * (enough for DeltaE*|dt| up to about 7000).  M is ignored by the EVOLVE
 * operations, Np by MOMENTS and MOMENTS_BACKWARD. */
gpuqt_status gpuqt_workspace_size(gpuqt_h h, int32_t op, int32_t B, int32_t M, int32_t Np,
                                  size_t *bytes);

/*
 * Chebyshev moments (Section 3.3):  mu[s][b][k] = <phiL_b| T_k(H/DeltaE_s) |phiR_b>
 * restricted to segment s, for k < M, by the recurrence of Section 3.2
 * (T_0 = 1, T_1 = H~, T_k = 2 H~ T_{k-1} - T_{k-2}).
 *   phiL, phiR : c128 [n][B] (may be the same pointer)
 *   mu         : c128 [n_segments][B][M], device
 * The reduction order is fixed, so repeated calls give bit-identical results.
 */
gpuqt_status gpuqt_moments(gpuqt_h h, int32_t B, const double *phiL, const double *phiR,
                           int32_t M, double *mu, void *ws, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): gpuqt_moments with its workspace in a fixed array
 * the library holds on every GPU it runs on (gpuqt_noalloc_scratch_bytes() bytes, 64 MiB), so
 * the call allocates nothing.  Same arguments, layouts and results as gpuqt_moments (bit for
 * bit under the same kernel variant), without ws / ws_bytes; GPUQT_ERR_WORKSPACE when
 * gpuqt_workspace_size(h, GPUQT_OP_MOMENTS, B, M, 0) exceeds the array (for B = 1, about
 * 4 x 16 n bytes plus the per-workgroup partials: n up to about 10^6).  All calls on one GPU
 * share that GPU's array: calls that overlap in time on one GPU (other streams, threads or
 * handles) race and must be serialised by the caller.  Nothing in the array needs to start
 * at zero; it keeps the last call's contents.
 */
gpuqt_status gpuqt_moments_noalloc(gpuqt_h h, int32_t B, const double *phiL, const double *phiR,
                                   int32_t M, double *mu, void *stream);
size_t gpuqt_noalloc_scratch_bytes(void);

/*
 * The same moments as gpuqt_moments by the one-moment-per-step recurrence of Sections 3.2-3.3
 * as the paper runs it: v_0 = phiR, v_1 = H~ v_0, v_k = 2 H~ v_{k-1} - v_{k-2}, mu_k = <phiL|v_k>,
 * M - 1 sparse steps whatever phiL and phiR are (gpuqt_moments needs about M/2 steps through
 * the product identities).  Same arguments, layouts, workspace (GPUQT_OP_MOMENTS) and errors
 * as gpuqt_moments; the fixed reduction order makes reruns bit-identical.  For comparisons
 * with the product-identity forms and for timing the single Chebyshev step.
 */
gpuqt_status gpuqt_moments_plain(gpuqt_h h, int32_t B, const double *phiL, const double *phiR,
                                 int32_t M, double *mu, void *ws, size_t ws_bytes, void *stream);

/*
 * Time evolution by the Chebyshev-Bessel series of Section 3.2:
 *   psi_out = U(dt) psi_in,  U(dt) = exp(-i H dt) for dt > 0 and exp(+i H |dt|) for dt < 0,
 *   U(+-dt) psi = sum_{m<Np} (2 - delta_m0) (-+i)^m J_m(DeltaE_s |dt|) T_m(H~) psi.
 * When chi_out is not NULL, also the commutator series of Section 3.2 combined
 * with the product rule:  chi_out = [X, U(dt)] psi_in + U(dt) chi_in
 * (chi_in NULL means zero), using [X, T_m] = 2[X,H~]T_{m-1} + 2H~[X,T_{m-1}] - [X,T_{m-2}].
 *   Np : terms; 0 = the smallest m > DeltaE|dt| with |J_m| < 1e-16 (max over segments)
 *   psi_in, chi_in, psi_out, chi_out : c128 [n][B]; outputs must not overlap inputs.
 */
gpuqt_status gpuqt_evolve(gpuqt_h h, int32_t B, double dt, int32_t Np, const double *psi_in,
                          double *psi_out, const double *chi_in, double *chi_out, void *ws,
                          size_t ws_bytes, void *stream);

enum { GPUQT_VELOCITY = 0, GPUQT_COMMUTATOR_XH = 1 };

/*
 * Velocity / commutator application (Section 4.2, velocity operator):
 *   GPUQT_VELOCITY      : out = V psi,     (V psi)_i     = i sum_j (x_j - x_i) H_ij psi_j
 *   GPUQT_COMMUTATOR_XH : out = [X,H] psi, ([X,H] psi)_i = -sum_j (x_j - x_i) H_ij psi_j
 * (x_j - x_i by minimum image when the segment is periodic).  Unscaled H.
 *   psi, out : c128 [n][B], must not overlap.
 */
gpuqt_status gpuqt_apply_commutator(gpuqt_h h, int32_t B, int32_t which, const double *psi,
                                    double *out, void *stream);

/*
 * VAC moments (Section 3.3, C_n^VAC):  for k < n_t,
 *   out[k][s][b][n] = Re <phi| U(t_k) V T_n(H~) U(t_k)^+ V |phi>,  t_k = dt[0] + ... + dt[k-1]
 * (row 0 at t = 0), computed as Re <V psi_L| T_n |psi_R> with psi_L = U(-t_k) phi and
 * psi_R = U(-t_k) V phi, advanced by U(-dt[k]) between rows.
 *   phi : c128 [n][B];  dt : HOST [n_t];  out : double [n_t][n_segments][B][M], device
 */
gpuqt_status gpuqt_vac(gpuqt_h h, int32_t B, const double *phi, int32_t n_t, const double *dt,
                       int32_t M, int32_t Np, double *out, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * MSD moments (Section 3.3, C_n^MSD):  for k < n_t,
 *   out[k][s][b][n] = Re <chi_{k+1}| T_n(H~) |chi_{k+1}>,  chi_{k+1} = [X, U(t_{k+1})] phi,
 *   t_{k+1} = dt[0] + ... + dt[k],
 * with chi advanced by the product rule chi_{k+1} = [X, U(dt_k)] psi_k + U(dt_k) chi_k,
 * psi_{k+1} = U(dt_k) psi_k, chi_0 = 0, psi_0 = phi.
 *   phi : c128 [n][B];  dt : HOST [n_t];  out : double [n_t][n_segments][B][M], device
 */
gpuqt_status gpuqt_msd(gpuqt_h h, int32_t B, const double *phi, int32_t n_t, const double *dt,
                       int32_t M, int32_t Np, double *out, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * Gradient of a loss on the Chebyshev moments of gpuqt_moments (Section 3.3):
 *   L = sum_{s,b,k} w[s][b][k] Re mu[s][b][k],  mu[s][b][k] = <phiL_b| T_k(H/DeltaE_s) |phiR_b>,
 * with DeltaE held fixed, with respect to
 *   - the on-site energies:   grad_onsite[i] += dL/dU_i,
 *   - the hopping classes:    grad_class[c]  += dL/ds_c, where s_c is the class scale of
 *                             gpuqt_update_h_values (class-c hoppings = s_c x their values
 *                             at build time; defined, and finite, at every s_c, also 0),
 *   - each stored hopping:    grad_hop[i][slot] += (dL/dRe H_ij, dL/dIm H_ij), entry `slot`
 *                             of row i of the neighbour list (j = nbr[i][slot]), every
 *                             entry an independent complex number (no Hermitian tie: see
 *                             gpuqt_tie_entry_gradient),
 * and optionally lam0 = sum_k w_k T_k(H~) phiL (the adjoint of phiR).
 * The entry gradient is sum_k f_k conj(lam_k)_i (v_{k-1})_j / DeltaE (f_1 = 1, else 2),
 * stored as (Re, -Im) of that sum.
 * Method: the recurrence of Section 3.2 run forwards with checkpoints of
 * (v_{js}, v_{js+1}) every s = ckpt_stride steps (0: ceil(sqrt(M))), then the
 * adjoint recurrence lam_k = w_k phiL + 2 H~ lam_{k+1} - lam_{k+2} run backwards,
 * recomputing each block of s forward vectors from its checkpoint.  ckpt_stride = 1
 * keeps every forward vector instead and reverses the two-chain form of the moments
 * (Section 3.3 moments by the product identities T_2k = 2 T_k T_k - T_0,
 * T_2k-1 = 2 T_k T_k-1 - T_1): chains a_k = T_k phiL, b_k = T_k phiR over
 * K = max(1, M/2) steps, both adjoint chains in one launch per step, about
 * 2K vectors of workspace and no recomputation; when phiL and phiR are the same
 * pointer the two chains coincide and only their adjoints' sum enters, so one
 * chain and one adjoint chain are run;
 * dL/dp = Re[ sum_{k>=2} 2 <lam_k| dH~/dp v_{k-1}> + <lam_1| dH~/dp v_0> ].
 * With grad_hop set the plain recurrence is reversed at every stride (ckpt_stride = 1
 * then keeps the M - 2 vectors v_1 .. v_{M-2}): the product identities hold for a
 * Hermitian H, which a change of one entry alone does not keep.
 *   phiL, phiR : c128 [n][B];  w : double [n_segments][B][M];  grad_onsite : double [n];
 *   grad_class : double [n_class] or NULL (at most 4 classes);
 *   grad_hop : double [n][max_nn][2] (max_nn of the descriptor) or NULL;
 *   lam0 : c128 [n][B] or NULL.  grad_class and grad_hop need grad_onsite.
 *   All device.  Workspace: gpuqt_workspace_size(h, GPUQT_OP_MOMENTS_BACKWARD, B, M,
 *   ckpt_stride) (its Np argument is the checkpoint stride).  Accumulation order is fixed:
 *   repeated calls give bit-identical gradients.
 */
gpuqt_status gpuqt_moments_backward(gpuqt_h h, int32_t B, const double *phiL, const double *phiR,
                                    int32_t M, const double *w, double *grad_onsite,
                                    double *grad_class, double *grad_hop, double *lam0,
                                    int32_t ckpt_stride, void *ws, size_t ws_bytes, void *stream);

/*
 * Gradient of a loss on the VAC moments of gpuqt_vac (Section 3.3, C_n^VAC; Section 2.2):
 *   L = sum_{k,s,b,n} w[k][s][b][n] out[k][s][b][n],  out as computed by gpuqt_vac,
 * with DeltaE held fixed, with respect to the on-site energies (grad_onsite[i] += dL/dU_i),
 * the hopping class scales (grad_class[c] += dL/ds_c as in gpuqt_moments_backward; s_c also
 * scales the velocity V = i[H, X] on those bonds) and each stored hopping (grad_hop as in
 * gpuqt_moments_backward, plus the velocity's share: V_ij = i dx_ij H_ij, so every
 * application a^+ V x adds i dx_ij conj(a_i) x_j to entry (i, j)).
 * Method: the forward VAC series (the states psi_L(t_k), psi_R(t_k) advanced by
 * U(-dt_k), Section 3.2), then the reverse over the rows: per row the adjoints of both
 * moment arguments (as gpuqt_moments_backward), back through phi_L = V psi_L (V is
 * Hermitian), and back through each evolution U(-dt) = sum_m c_m T_m(H~) by the reverse
 * recurrence with sources conj(c_m) g, whose lam_0 is U(+dt) g.
 *   ckpt_stride 0: the moment and evolution reverses recompute forward vectors from
 *   checkpoints every ceil(sqrt(L)) steps (L = max(M, Np)); 1: every forward vector is
 *   kept and each row's moments are reversed in the two-chain form (one pass gives both
 *   adjoints and the parameter terms); needs about L vectors more workspace.
 *   time_stride 1: every state psi_L(t_k), psi_R(t_k) is kept (2 n_t - 1 vectors);
 *   s >= 2: only the states of rows 0, s, 2s, ... are kept and each segment of s rows is
 *   re-evolved from its checkpoint when the reverse reaches it (2 ceil(n_t / s) - 1 +
 *   2 (s - 1) vectors, one more forward evolution of every step); 0: s = ceil(sqrt(n_t))
 *   (1 when that is n_t).  The gradients agree to rounding whatever the strides.
 *   phi : c128 [n][B];  dt : HOST [n_t];  w : double [n_t][n_segments][B][M];
 *   grad_onsite : double [n];  grad_class : double [n_class] or NULL (at most 4 classes);
 *   grad_hop : double [n][max_nn][2] or NULL (with it, the rows' moments are reversed by
 *   the plain recurrence also at ckpt_stride 1).
 *   Workspace: gpuqt_vac_backward_workspace_size with the same strides.
 */
gpuqt_status gpuqt_vac_backward(gpuqt_h h, int32_t B, const double *phi, int32_t n_t,
                                const double *dt, int32_t M, int32_t Np, const double *w,
                                double *grad_onsite, double *grad_class, double *grad_hop,
                                int32_t ckpt_stride, int32_t time_stride, void *ws, size_t ws_bytes,
                                void *stream);

/*
 * Hermitian tie of per-entry gradients (of gpuqt_moments_backward / gpuqt_vac_backward).
 * A Hermitian H stores each bond h = H_ij = conj(H_ji) twice; the gradient of L with
 * respect to (Re h, Im h) is the sum of the two entries' gradients with the sign of the
 * Im part flipped on the partner:
 *   tied[i][s] = (g[i][s].re + g[j][p].re, g[i][s].im - g[j][p].im),
 * where entry s of row i points to j and p is its partner in row j: the q-th entry of
 * row j that points to i when s is the q-th entry of row i that points to j.  An entry
 * without a partner, and every padding slot, is copied.  Each bond's value then sits at
 * both of its entries (the partner holding (re, -im)).
 *   untied, tied : double [n][max_nn][2], device, distinct buffers (no in-place).
 * Enqueued on `stream`; GPUQT_ERR_ARG for NULL, equal or misaligned pointers.
 */
gpuqt_status gpuqt_tie_entry_gradient(gpuqt_h h, const double *untied, double *tied, void *stream);

/* Workspace bytes of gpuqt_vac_backward (dt: HOST [n_t], needed for the automatic Np). */
gpuqt_status gpuqt_vac_backward_workspace_size(gpuqt_h h, int32_t B, int32_t n_t, const double *dt,
                                               int32_t M, int32_t Np, int32_t ckpt_stride,
                                               int32_t time_stride, size_t *bytes);

/*
 * Recorded VAC forward, for a backward pass that recomputes nothing (the
 * forward of Section 3.3's VAC rows already produces every vector the reverse
 * needs; these calls keep them instead of overwriting them).
 * gpuqt_vac_record computes the same rows as gpuqt_vac (same arguments,
 * workspace and results, bit for bit) and also writes into `tape` (device,
 * caller-owned, at least gpuqt_vac_tape_size bytes, 16-byte aligned) the states
 * psi_L(t_k), psi_R(t_k), per row both moment chains T_j V psi_L(t_k) and
 * T_j psi_R(t_k) of the product-identity form (j = 1 .. max(1, M/2)), and per
 * time step both evolution chains T_m psi_L(t_k), T_m psi_R(t_k) (m = 1 .. P-1,
 * P the largest number of terms over the steps): (2 n_t - 1 + n_t * 2 *
 * max(1, M/2) + (n_t - 1) * 2 (P - 1)) vectors of n x B complex128.
 * gpuqt_vac_backward_tape then gives the gradients of gpuqt_vac_backward
 * (same arguments, results to rounding) from that tape, skipping the
 * re-evolution of the states and every forward chain; the tape must come from
 * gpuqt_vac_record with the same handle values, B, phi, dt, M and Np.
 * Workspace: gpuqt_vac_backward_tape_workspace_size.
 * GPUQT_ERR_WORKSPACE for a tape or workspace that is too small.
 */
gpuqt_status gpuqt_vac_tape_size(gpuqt_h h, int32_t B, int32_t n_t, const double *dt, int32_t M,
                                 int32_t Np, size_t *bytes);
gpuqt_status gpuqt_vac_record(gpuqt_h h, int32_t B, const double *phi, int32_t n_t, const double *dt,
                              int32_t M, int32_t Np, double *out, void *ws, size_t ws_bytes,
                              void *tape, size_t tape_bytes, void *stream);
gpuqt_status gpuqt_vac_backward_tape(gpuqt_h h, int32_t B, const double *phi, int32_t n_t,
                                     const double *dt, int32_t M, int32_t Np, const double *w,
                                     double *grad_onsite, double *grad_class, const void *tape,
                                     size_t tape_bytes, void *ws, size_t ws_bytes, void *stream);
gpuqt_status gpuqt_vac_backward_tape_workspace_size(gpuqt_h h, int32_t B, int32_t n_t,
                                                    const double *dt, int32_t M, int32_t Np,
                                                    size_t *bytes);

/*
 * Choose the sparse-kernel variant for this handle by measurement: times 12
 * Hermitian moment steps (Section 3.2 recurrence on a scratch vector) of each
 * variant and keeps the fastest for all later calls on the handle.  Variant
 * bit 0: non-temporal loads of the once-read streams; bit 1: the banded row
 * order (built when a segment's row period D would make the window between
 * the first and last use of a gathered element exceed about 2.5 MiB of
 * streamed data at this B, and for B >= 2 with two bands per period for
 * periods of 1024 rows or more: workgroups then sweep bands of W rows of the
 * period one period after another, so rows D apart are visited W rows apart);
 * bit 26: on a periodic simple cubic box (one segment, rows x + Lx (y + Ly z), each
 * with its six periodic neighbours, one uniform hopping; gpuqt_h_info_t.box), the Hermitian
 * moment step of blocks of B >= 2 vectors as a box stencil: a workgroup marches through
 * a column of the box, keeps each lane's elements of three consecutive planes in
 * registers and the current plane's tile in LDS, so x is read about once per step instead
 * of once per neighbour and no neighbour indices are read (timed against the best other
 * variant, kept when faster); on segments that are all periodic squares
 * (gpuqt_h_info_t.sheets) bit 26 selects the two-dimensional form: a workgroup marches
 * along y through a strip of 256 / B cells of one segment, rows y - 1, y, y + 1 in
 * registers and row y in LDS; bit 27: the fused MSD term likewise (both chains staged,
 * where the position differences are +-dx on the x neighbours and 0 on the others,
 * gpuqt_h_info_t.box_msd), timed against the MSD family's best and kept when faster;
 * both box kernels are timed uncapped and at caps 1..6 and keep the fastest as their
 * family's own cap;
 * bit 6 (with bit 1): the pencil order instead (built for segments with a row
 * period of at least 128 rows: the four wavefronts of a workgroup take the
 * same rows of four consecutive periods at once, so a row's neighbours one
 * period away are the rows a sibling wavefront on the same compute unit is
 * loading, and the L1 serves them);
 * bits 2-5: a cap on resident workgroups per compute unit (0: as many as the
 * kernel's registers allow).  Each of the four load/order variants is timed
 * uncapped and at every cap of 2..6 below its occupancy limit: fewer waves in
 * flight shrink the window of rows whose gathered elements must stay cached,
 * which can outweigh the lost latency hiding.  The cap applies to every
 * kernel family on the handle; then, at the chosen load variant, the
 * two-chain moment step, the two-vector evolution term and the MSD term are
 * each timed at the same caps and get their own (kernel_variant bits 8-25),
 * the two series terms also with the other load variant (bit 7 when that is
 * faster for the pair of them).
 * Synchronises the stream.
 *   ws : device workspace of gpuqt_workspace_size(h, GPUQT_OP_AUTOTUNE, B, 0, 0) bytes
 *        (eight vectors); one of three vectors plus the partial sums tunes the
 *        Hermitian step only.
 *   times_us : NULL or HOST [7], microseconds per step of load/order variants 0..3, of
 *              the pencil order with plain (4) and non-temporal (5) loads, each at its best
 *              cap, and of the periodic-box stencil (6, at the chosen cap); 0 for what this
 *              handle and B do not have.
 * Not safe while other calls on the handle are in flight.
 */
gpuqt_status gpuqt_autotune(gpuqt_h h, int32_t B, void *ws, size_t ws_bytes, void *stream,
                            double *times_us);

/* Set the kernel variant without measuring, with the bits of gpuqt_h_info_t.kernel_variant:
 * load variant in bits 0-1, per-CU cap 0..8 in bits 2-5, the pencil order in bit 6 (with
 * bit 1), in bit 7 the series families (evolution and MSD terms) on the other load variant
 * than bit 0, and from bit 8 three bits per kernel family (0: the per-CU cap, 1 + c:
 * cap c of 0..6), so a code read from gpuqt_h_info after gpuqt_autotune reproduces the tuned
 * configuration.  The banded and pencil bits only take effect for block widths that have
 * such an order (gpuqt_h_info_t.banded_mask, pencil_mask); a pencil bit for a width without
 * a pencil order falls back to the banded order.  Bit 26 (the box stencil of the Hermitian
 * step) takes effect on a periodic box (gpuqt_h_info_t.box) for blocks of B >= 2, bit 27
 * (that of the MSD term) where gpuqt_h_info_t.box_msd is also set.
 * GPUQT_ERR_ARG for a negative code, a per-CU cap above 8, bit 6 without bit 1 or bits set
 * above bit 27. */
gpuqt_status gpuqt_set_variant(gpuqt_h h, int32_t variant);

/*
 * Tuning cache (process-wide, thread-safe).  A kernel variant measured by gpuqt_autotune is
 * kept under a key of everything the choice depends on: the device architecture, the
 * orbital count (log2 bucket), the row structure (fixed width K or widest slice, slice
 * height), the hopping storage, the segment count, the row period (log2 bucket), which
 * block widths have a banded row order, and B (gpuqt_tune_cache_key writes it, at most
 * len bytes with the terminating NUL).
 * gpuqt_autotune_cached applies the cached code for the handle's key, or runs
 * gpuqt_autotune (same arguments) and caches its choice; *from_cache (may be NULL) tells
 * which.  A cached code leaves times_us zero and needs no workspace (ws may be NULL then).
 * gpuqt_tune_cache_load merges a text file of "<key>TAB<code>" lines ('#' starts a
 * comment line; GPUQT_ERR_ARG if it cannot be opened, GPUQT_ERR_LAYOUT with file:line for a
 * malformed line, nothing merged then); gpuqt_tune_cache_save writes every entry.
 */
gpuqt_status gpuqt_tune_cache_key(gpuqt_h h, int32_t B, char *buf, size_t len);
gpuqt_status gpuqt_autotune_cached(gpuqt_h h, int32_t B, void *ws, size_t ws_bytes, void *stream,
                                   double *times_us, int32_t *from_cache);
gpuqt_status gpuqt_tune_cache_load(const char *path);
gpuqt_status gpuqt_tune_cache_save(const char *path);
void gpuqt_tune_cache_clear(void);

/*
 * Block width for n_vectors independent random vectors (Section 4.2.7: the random vectors
 * are independent, so they may be advanced in blocks of B columns sharing each matrix read):
 * for every B in {1, 2, 4, 8, 16} with B <= n_vectors whose autotuning workspace
 * (gpuqt_workspace_size(h, GPUQT_OP_AUTOTUNE, B, 0, 0)) fits in ws_bytes, autotunes the
 * handle at B (caching each choice) and measures the Hermitian moment step; writes the B
 * with the least time per vector and step to *best_B, the microseconds per vector-step of
 * each width to us_per_vector_step (HOST [5], index log2 B, 0 where not tried; may be NULL),
 * and leaves the handle tuned for best_B.  Synchronises the stream.
 */
gpuqt_status gpuqt_autotune_block(gpuqt_h h, int32_t n_vectors, void *ws, size_t ws_bytes, void *stream,
                                  int32_t *best_B, double *us_per_vector_step);

/*
 * gpuqt_build_h with the sliced-ELL slice height chosen by measurement: the layout of desc
 * (its slice_height ignored) is built at heights 32, 64, 128 and 256, each autotuned at
 * block width B (allocating and freeing its own autotuning workspace), and the handle whose
 * Hermitian moment step is fastest is returned in *out (the others are destroyed).
 * *slice_height (may be NULL) receives its height, us_per_step (HOST [4] or NULL) the best
 * microseconds per step at each height.  Errors as gpuqt_build_h, plus GPUQT_ERR_NOMEM when
 * a workspace cannot be allocated.
 */
gpuqt_status gpuqt_build_h_tuned(const gpuqt_h_desc *desc, int32_t B, void *stream, gpuqt_h *out,
                                 int32_t *slice_height, double *us_per_step);

/*
 * KPM reconstruction (Section 3.3, same prefactor for DOS, rho*C_vv, rho*DeltaX^2):
 *   out[r][e] = 2 / (pi Omega DeltaE sqrt(1 - E~^2)) sum_{n<M} g_n (2 - delta_n0) T_n(E~) C[r][n],
 *   E~ = energies[e] / DeltaE, g_n the Jackson damping (jackson != 0) or 1.
 *   C : double [R][M], energies : double [n_E], out : double [R][n_E]; all device.
 * The expansion only exists inside the scaled band: out is NaN where |E~| >= 1
 * (the energies live on the device, so this is not checked on the host).
 */
gpuqt_status gpuqt_kpm_reconstruct(int32_t R, int32_t M, const double *C, int32_t n_E,
                                   const double *energies, double energy_max, double volume,
                                   int32_t jackson, double *out, void *stream);

/* Running electrical conductivity (Section 2.2, e = 1) from KPM-reconstructed rows:
 *   GPUQT_SIGMA_VAC: y[k][e] = rho C_vv(E_e, t_k) at the VAC row times t_k = sum_{j<k} dt_j;
 *     sigma[k][e] = int_0^{t_k} rho C_vv dt by the trapezoid rule over the rows (sigma[0] = 0).
 *   GPUQT_SIGMA_MSD: y[k][e] = rho DeltaX^2(E_e, t_{k+1}) at the MSD row times
 *     t_{k+1} = sum_{j<=k} dt_j, with DeltaX^2 = 0 at t = 0; sigma[k][e] = (y_k - y_{k-1}) / (2 dt_k),
 *     the slope of the straight line between consecutive rows halved, which belongs to the
 *     midpoint t_{k+1} - dt_k / 2 (NaN where dt_k = 0).
 *   dt : double [n_t], y and sigma : double [n_t][n_E]; all device; sigma must not overlap y.
 */
enum { GPUQT_SIGMA_VAC = 0, GPUQT_SIGMA_MSD = 1 };
gpuqt_status gpuqt_running_conductivity(int32_t mode, int32_t n_t, const double *dt, int32_t n_E,
                                        const double *y, double *sigma, void *stream);

/* Transport regimes (Section 2.2, e = hbar = 1) per energy from reconstructed rows:
 *   sigma_sc[e] = max over the rows k of sigma[k][e], the semiclassical conductivity taken, as
 *                 in the paper, as the maximum of the running conductivity (NaN rows skipped);
 *   v[e]   = sqrt(C_vv(E_e, 0)), the group velocity, C_vv(E, 0) = vac0[e] / rho[e];
 *   tau[e] = sigma_sc / (rho v^2), the relaxation time (equation sigma_sc);
 *   mfp[e] = v tau, the mean free path (equation mfp);
 *   L[k][e] = 2 sqrt(DeltaX^2(E_e, t)), DeltaX^2 = msd[k][e] / rho[e] (equation L);
 *   xi[e]  = L[n_t - 1][e] / (2 pi), the localization length, the last row standing for
 *            t -> infinity (equation xi).
 * rho : double [n_E] (the DOS of gpuqt_kpm_reconstruct); vac0 : [n_E] the VAC row at t = 0
 * (rho C_vv), or NULL; sigma : [n_t][n_E] a running conductivity (gpuqt_running_conductivity),
 * or NULL; msd : [n_t][n_E] rho DeltaX^2 rows, or NULL.  Outputs may be NULL; each one needs
 * its inputs (sigma_sc: sigma; v: vac0; tau, mfp: sigma and vac0; L, xi: msd), must not overlap
 * them, and is NaN where rho <= 0, C_vv(E, 0) < 0 (v), rho v^2 <= 0 (tau, mfp) or
 * DeltaX^2 < 0 (L, xi).  All device; stream-ordered.
 */
gpuqt_status gpuqt_transport_lengths(int32_t n_t, int32_t n_E, const double *rho, const double *vac0,
                                     const double *sigma, const double *msd, double *sigma_sc,
                                     double *v, double *tau, double *mfp, double *L, double *xi,
                                     void *stream);

/* Transpose of gpuqt_kpm_reconstruct (for gradients of losses on the reconstructed
 * functions): out[r][n] = sum_e g[r][e] * d out_kpm[r][e] / d C[r][n], energies with
 * |E~| >= 1 contributing nothing.  g : double [R][n_E], energies : double [n_E],
 * out : double [R][M]; all device. */
gpuqt_status gpuqt_kpm_reconstruct_adjoint(int32_t R, int32_t M, const double *g, int32_t n_E,
                                           const double *energies, double energy_max, double volume,
                                           int32_t jackson, double *out, void *stream);

/* Measurement: kernel families whose runs of launches gpuqt_timing reports. */
enum {
  GPUQT_K_MOMENT = 0,       /* plain moment step (recomputation, autotuning) */
  GPUQT_K_MOMENT_SYM = 1,   /* moment step of a Hermitian set (phiL = phiR) */
  GPUQT_K_MOMENT_PAIR = 2,  /* moment step with two chains (phiL != phiR) */
  GPUQT_K_EVOLVE = 3,       /* evolution series term */
  GPUQT_K_MSD = 4,          /* fused evolution + commutator series term */
  GPUQT_K_EVOLVE_PAIR = 5,  /* evolution series term on two vectors (the VAC states) */
  GPUQT_K_COUNT = 6
};

/* enable != 0: every later compute call on the handle records a HIP event before and after
 * each uninterrupted run of launches of one kernel family, on the call's stream (calls on a
 * stream that is being captured into a graph record nothing).  The events are released by
 * gpuqt_timing or gpuqt_destroy_h.  Not thread-safe: one host thread per handle. */
gpuqt_status gpuqt_set_timing(gpuqt_h h, int32_t enable);

/* Waits for the recorded events and returns, per family, the summed milliseconds of its
 * runs (ms[GPUQT_K_COUNT], HOST) and the number of launches they held
 * (launches[GPUQT_K_COUNT], HOST); then forgets the records. */
gpuqt_status gpuqt_timing(gpuqt_h h, double *ms, int64_t *launches);

/* Host helpers (no device use). */

/*
 * Input folder of the paper's program (Section 4.2), read on the host:
 *   neighbour.in  "N max_nn", then per site "count j_1 j_2 ..." (required)
 *   hopping.in    "real" or "complex", then per site the hoppings of its neighbours in
 *                 neighbour.in order (complex: re im pairs); absent: every hopping is -1
 *   potential.in  one on-site energy per site; absent: 0
 *   position.in   "length_x volume", then one coordinate per site (required)
 *   energy.in     count, then the energies (required)
 *   time_step.in  count, then the time steps (required when VAC or MSD is asked for)
 *   para.in       keywords calculate_vac, calculate_msd, number_of_random_vectors N_r,
 *                 number_of_moments N_m, energy_max DeltaE; defaults N_r = 1,
 *                 N_m = 1000, DeltaE = 10 (Section 4.2.7)
 * gpuqt_model_load returns GPUQT_ERR_ARG for a missing required file and
 * GPUQT_ERR_LAYOUT with file:line for malformed contents.  The model owns its arrays;
 * gpuqt_model_desc fills a descriptor pointing into them (valid until gpuqt_model_free).
 */
typedef struct gpuqt_model_s *gpuqt_model;
typedef struct {
  int32_t n_random_vectors;
  int32_t n_moments;
  double energy_max;
  int32_t calculate_vac;
  int32_t calculate_msd;
  int32_t n_energies;
  int32_t n_time_steps;
  const double *energies;    /* HOST [n_energies], owned by the model */
  const double *time_steps;  /* HOST [n_time_steps] or NULL, owned by the model */
} gpuqt_model_params_t;
gpuqt_status gpuqt_model_load(const char *dir, gpuqt_model *out);
gpuqt_status gpuqt_model_desc(gpuqt_model m, gpuqt_h_desc *d);
gpuqt_status gpuqt_model_params(gpuqt_model m, gpuqt_model_params_t *p);
void gpuqt_model_free(gpuqt_model m);

/* The row schedule of the sparse kernels, as the library plans it for `cus` compute units
 * and block width B (introspection; the kernels enumerate rows with the same host/device
 * rule): segments seg_offsets (HOST [n_segments+1], from 0, ascending), row period per
 * segment (HOST [n_segments] or NULL: plain order), band width band_rows (multiple of 64;
 * segments whose period exceeds it take the banded order; with pencil != 0 every segment
 * whose period is at least 128 rows takes the pencil order of that band width instead, as
 * gpuqt_autotune's bit 6 describes).  Writes for every row the
 * logical workgroup that visits it (block_of_row, HOST int32 [n]) and the workgroup's
 * iteration at that visit (iter_of_row, HOST int32 [n]); -1 for a row no workgroup visits.
 * GPUQT_ERR_LAYOUT if some row would be visited twice. */
gpuqt_status gpuqt_schedule_rows(int32_t n_segments, const int64_t *seg_offsets, const int64_t *period,
                                 int32_t band_rows, int32_t pencil, int32_t cus, int32_t B,
                                 int32_t *block_of_row, int32_t *iter_of_row);

/* Jackson damping g_n, n < M (Section 3.3):  g_n = (1 - n a) cos(pi n a) + a sin(pi n a) cot(pi a),
 * a = 1/(M+1).  g: HOST [M]. */
gpuqt_status gpuqt_jackson(int32_t M, double *g);

/* Bessel functions of the first kind J_m(tau), m < Np, tau >= 0: the coefficients of the
 * Chebyshev expansion of the evolution operator, U(dt) = sum_m (2 - delta_m0) (-i)^m
 * J_m(DeltaE dt) T_m(H~) (Section 3.2, the first Chebyshev expansion), evaluated by Miller's
 * backward recurrence normalised by J_0 + 2 sum_k J_2k = 1.  J: HOST [Np].
 * GPUQT_ERR_ARG for tau < 0 or not finite, Np < 0, or J NULL with Np > 0. */
gpuqt_status gpuqt_bessel(double tau, int32_t Np, double *J);

/* Number of Chebyshev terms for U(dt): the smallest m > tau with |J_m(tau)| < 1e-16,
 * tau = DeltaE |dt| (Section 3.2: up to machine precision, proportional to dt).
 * Returns -1 for tau < 0 or not finite. */
int32_t gpuqt_auto_terms(double tau);

/* Message of the last failure in this thread ("" if none). */
const char *gpuqt_last_error(void);

/* Measurement helper: copy `bytes` (multiple of 16) from src to dst on the
 * device with the same 16-byte vector loads the sparse steps use; its
 * duration gives the attainable HBM bandwidth.  src, dst: device, no overlap. */
gpuqt_status gpuqt_copy_probe(const void *src, void *dst, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GPUQT_H */
