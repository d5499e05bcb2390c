/*
 * mrtlb.h -- C ABI of the MI355X (gfx950) Hermite-matrix MRT lattice
 * Boltzmann library.
 *
 * The library runs the per-time-step fused collide-and-stream of the unified
 * MRT-LB method of Shi, Yuan & Chai (arXiv 2512.16230) on multispeed
 * rectangular lattices: the update of eq. (2-3) (theta = gamma = 1, full
 * correction) with the Hermite-space collision of eq. (H-MRT-LB), the
 * generalized third-order equilibrium of eq. (feq-1), the auxiliary moments
 * M30 / M2G for the Navier-Stokes equations (Sec. III) and M20 / M1G for the
 * nonlinear convection-diffusion equation (App. A), and propagation along
 * the rD2Q25, rD2Q13, rD3Q53 and rD3Q33 velocity sets (Sec. V, App. D).
 *
 * Conventions shared by every entry point
 *  - Every call returns an mrtlb_status (0 = success, < 0 = error) and never
 *    throws; mrtlb_last_error() returns a thread-local message describing the
 *    last failure on the calling thread.
 *  - Host arrays are borrowed for the duration of the call only, are FP64,
 *    and are laid out structure-of-arrays with x fastest: a scalar field has
 *    N = nx*ny*nz entries at index (z*ny + y)*nx + x; a vector field of
 *    dimension d is d consecutive scalar fields (component-major); a
 *    population array is b consecutive scalar fields, population j in the
 *    lattice's velocity order (mrtlb_lattice_query).
 *  - Device memory belongs to the library and is released by the matching
 *    destroy call.  All device work of a solve is enqueued on the stream given
 *    to mrtlb_ctx_create (borrowed; e.g. a PyTorch stream); calls that return
 *    host data synchronize that stream first.
 *  - Periodic boundaries in every direction; dt = 1 and dx_a = c_a (lattice
 *    units).
 *  - Handles are not thread-safe: one thread at a time per context.
 */
#ifndef MRTLB_H
#define MRTLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MRTLB_OK = 0,
  MRTLB_EINVAL = -1,   /* bad argument: null pointer, size, enum, rates    */
  MRTLB_ENOMEM = -2,   /* footprint over the context's HBM budget, or a
                          device allocation failed; nothing is allocated  */
  MRTLB_EDEVICE = -3,  /* a HIP runtime call failed                        */
  MRTLB_ENUMERIC = -4  /* a weight <= 0, singular Hermite Gram matrix, or a
                          non-finite value found in a solve's state         */
} mrtlb_status;

typedef struct mrtlb_ctx mrtlb_ctx;
typedef struct mrtlb_lattice mrtlb_lattice;
typedef struct mrtlb_solve mrtlb_solve;

/* Message of the last failed call on this thread ("" if none). */
const char* mrtlb_last_error(void);

/* ABI version, (major << 16) | minor. */
int mrtlb_version(void);

/* Page-locked host memory from the library's HIP runtime, for staging the
 * host arrays of mrtlb_init_fields / mrtlb_read_moments (copies from and to
 * it run at DMA speed).  The caller owns it; release with mrtlb_host_free.
 * Errors: EINVAL (NULL out, bytes == 0), ENOMEM. */
mrtlb_status mrtlb_host_alloc(size_t bytes, void** out);
void mrtlb_host_free(void* p);

/* ---------------------------------------------------------------------------
 * Context: one device, one stream, one HBM budget.
 *   device            HIP device ordinal.
 *   stream            hipStream_t to enqueue on (borrowed, may be NULL for the
 *                     default stream).
 *   hbm_budget_bytes  upper bound on the device memory all solves of this
 *                     context may hold; 0 = 90% of the device's free memory.
 * ------------------------------------------------------------------------- */
mrtlb_status mrtlb_ctx_create(int device, void* stream, size_t hbm_budget_bytes, mrtlb_ctx** out);
void mrtlb_ctx_destroy(mrtlb_ctx* ctx);
/* Bytes held by the context's solves and the budget. */
mrtlb_status mrtlb_ctx_memory(const mrtlb_ctx* ctx, size_t* used, size_t* budget);
/* Block until all work enqueued by the context has finished. */
mrtlb_status mrtlb_ctx_synchronize(mrtlb_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Lattice (host only, FP64).  Velocity sets and weights follow the paper:
 *   MRTLB_RD2Q25  Sec. V eq. (3-1), weights eq. (WeightQ25), free weights
 *                 free_w = {w13, w17, w18, w21}.
 *   MRTLB_RD2Q13  Sec. V eq. (Q13lattice), closed-form weights, no free w.
 *   MRTLB_RD3Q53  App. D, weights with free_w = {w33, w37, w41, w45}
 *                 (d0a = cs^2 / c_a^2).
 *   MRTLB_RD3Q33  App. D, weights unique for a given cs^2, no free w.
 *   MRTLB_RD2Q21  the rD2Q25 subgroup without the (+-3, +-3) velocities
 *                 (Sec. V item (i): w21 = 0), the first 21 columns of
 *                 eq. (3-1); free_w = {w13, w17, w18}.
 *   MRTLB_D2Q21K  App. C, the D2Q21 with knight-move velocities (+-2, +-1),
 *                 (+-1, +-2) and (+-3, 0), (0, +-3) (not an rD2Q25
 *                 subgroup); free_w = {w9}.
 *   MRTLB_RD3Q45  the rD3Q53 subgroup without the (+-2, +-2, +-2) velocities
 *                 (w45 = 0), the first 45 columns of the App. D velocity
 *                 matrix; free_w = {w33, w37, w41}.
 *   MRTLB_RD2Q17_1 .. MRTLB_RD2Q17_5  App. C, D2Q17 cases 1-5 in their printed
 *                 velocity order: rD2Q25 subgroups.  free_w = {w13, w17, w18,
 *                 w21} of eq. (WeightQ25); with the given c and cs2 the weights
 *                 of the case's dropped velocity groups must vanish (|w| <=
 *                 1e-12, else EINVAL).
 *   MRTLB_D2Q9, MRTLB_D3Q27  standard single-layer lattices (the first layer
 *                 of eq. (3-1) / of the App. D velocity matrix) for the
 *                 k = 1 model of the standard-lattice case (Sec. IV-B):
 *                 weights prod_a (1 - d_a at rest, d_a / 2 at +-1),
 *                 d_a = cs^2 / c_a^2 (the moment conditions of Sec. V a
 *                 single layer can meet); no free w.  These lattices have no
 *                 pure third-order rows, and their normal second-order rows
 *                 relax with the non-diagonal S2 block of eqs. (4-27),
 *                 (4-27-1) (see mrtlb_model_desc).  Use m30 = 0 (M30 = 0
 *                 there).  The NCDE and CDE models run on D2Q9 too.
 * c[0..d-1] = c_a = dx_a/dt; cs2 = sound speed squared (direction
 * independent, Remark 2).  The Hermite rows of orders 0..3 are
 * H0 = 1, H1 = c, H2 = cc - cs^2 I, H3 = c_a(c_b^2 - cs^2), c_x c_y c_z and
 * c_a(c_a^2 - 3 cs^2) minus its W-projection on span{c_a(c_b^2 - cs^2)}
 * (eq. CorrectQ25 and its App. D analogue).
 * Errors: EINVAL (unknown kind, c <= 0, cs2 <= 0, wrong n_free),
 *         ENUMERIC (some weight <= 0 or a singular correction system).
 * ------------------------------------------------------------------------- */
typedef enum { MRTLB_RD2Q25 = 0, MRTLB_RD2Q13 = 1, MRTLB_RD3Q53 = 2, MRTLB_RD3Q33 = 3, MRTLB_RD2Q21 = 4,
               MRTLB_D2Q21K = 5, MRTLB_RD3Q45 = 6, MRTLB_RD2Q17_1 = 7, MRTLB_RD2Q17_2 = 8, MRTLB_RD2Q17_3 = 9,
               MRTLB_RD2Q17_4 = 10, MRTLB_RD2Q17_5 = 11, MRTLB_D2Q9 = 12, MRTLB_D3Q27 = 13,
               MRTLB_CUSTOM = 14 } mrtlb_lattice_kind;

typedef struct {
  int kind;          /* mrtlb_lattice_kind */
  double c[3];       /* c_a; c[2] ignored in 2D */
  double cs2;
  double free_w[4];  /* free weights, see above */
  int n_free;        /* 4 for RD2Q25 and RD3Q53, 0 otherwise */
  /* MRTLB_CUSTOM only (ignored otherwise): dimension d (2 or 3), b
   * velocities (b <= 53) given as integer multiples e (b*d ints, |e| <= 8,
   * row j = velocity j) and their weights w (b doubles, positive, summing
   * to 1); both arrays are copied.  The Hermite rows are built as for the
   * multispeed lattices (corrected pure third-order rows) and must come out
   * W-orthogonal with nonzero norms, else ENUMERIC.  Solves on a custom
   * lattice run run-time-generic kernels (one node per thread, every
   * population read twice per step) and take the NSE models only. */
  int d, b;
  const int* e;
  const double* w;
} mrtlb_lattice_desc;

mrtlb_status mrtlb_lattice_create(const mrtlb_lattice_desc* desc, mrtlb_lattice** out);
void mrtlb_lattice_destroy(mrtlb_lattice* lat);
/* Query: b, d, e (b*d ints, integer multiples, row j = velocity j), w (b),
 * nlow (number of Hermite rows of order <= 3: 10 in 2D, 20 in 3D; 8 and 17
 * on the standard lattices, which have no pure rows),
 * H (nlow*b, row-major, component rows 1, x, y, [z], xx, yy, [zz], xy, [xz, yz],
 * then x yy, [x zz], y xx, [y zz], [z xx, z yy], [xyz], xxx, yyy, [zzz] with the
 * pure rows corrected) and norms (nlow) = H_r W H_r^T.  Any output pointer
 * may be NULL. */
mrtlb_status mrtlb_lattice_query(const mrtlb_lattice* lat, int* b, int* d, int* e, double* w, int* nlow,
                                 double* H, double* norms);

/* ---------------------------------------------------------------------------
 * Model.  Relaxation rates are the diagonal of S in Hermite space:
 *   s0 (order 0), s1 (order 1), s_shear (off-diagonal and deviatoric normal
 *   order-2 rows), s_bulk (trace of order 2), s3 (order 3), s_high (every
 *   row above order 3).  Shear viscosity nu = cs^2 (1/s_shear - 1/2) dt,
 *   bulk nu_b = (2/d) cs^2 (1/s_bulk - 1/2) dt (eq. 4-29, k = 0).
 *   On the standard lattices (k = 1) the same nu and nu_b fix the normal
 *   block S2 = (diag(1/s_sa) + a b^T / d)^-1 of eqs. (4-27), (4-27-1):
 *   1/s_sa = 1/2 + 2 nu / (c_a^2 - cs^2), 1/s_ba = 1/2 + d nu_b / (c_a^2 - cs^2),
 *   a_a = (1/s_ba - 1/s_sa)(c_a^2 - cs^2), b_b = 1 / (c_b^2 - cs^2) (eq. 4-29
 *   with k = 1); the off-diagonal rows keep s_shear.  The auxiliary
 *   second moment uses the same (I - S2/2).
 * MRTLB_NSE_INC   M0 = rho_bar, M1 = rho0 u, M2 = rho0 uu + cs^2 rho_bar I,
 *                 M3 = rho0 cs^2 Delta.u + M30 (Sec. III, multispeed case);
 *                 rho_bar carries the pressure p = cs^2 rho_bar.
 * MRTLB_NSE_COMP  isothermal compressible: M0 = rho, M1 = rho u,
 *                 M2 = rho uu + p I, M3 = p Delta.u + M30, p = cs^2 rho.
 *   Both: M30 = rho uuu when m30 != 0; a body force F enters as
 *   M1F = F (eq. M-NSEs-5) with the auxiliary
 *   M2G = (I - S2/2)(uF + Fu) (eq. M2G-1, S = 0); u = (sum c f + F/2)/rho.
 * MRTLB_NCDE      phi_t + div(phi u) = div(D(phi) grad phi),
 *                 D = D0 (1 + D2 phi^2), constant advection adv_u:
 *                 M0 = phi, M1 = phi u, M2 = cs^2 Phi(phi) I + phi uu,
 *                 K Phi' = D with K = cs^2 (1/s1 - 1/2), and the auxiliary
 *                 first moment (I - S1/2) u [(phi^n - phi^{n-1}) +
 *                 u . grad phi^{n-1}] (eq. M-NCDE-6, case (1); central
 *                 differences, phi^{-1} = phi^0).
 * MRTLB_CDE       phi_t + u . grad phi = div(K grad phi) with a velocity
 *                 field u(x) given per node (the NCDE special case (3)):
 *                 diffusion-type equilibrium M0 = phi, M1 = 0,
 *                 M2 = cs^2 phi I, M3 = 0; source S_G = -u . grad phi with
 *                 grad phi = -s1 sum_j c_j f_j / cs^2 and
 *                 phi = sum_j f_j + S_G / 2 (eq. M-NCDE-3-00),
 *                 M0G = (1 - s0/2) S_G; K = cs^2 (1/s1 - 1/2).  The velocity field
 *                 may change between steps (mrtlb_set_velocity_field).
 *   The NCDE and CDE run on every compiled lattice, 2D and 3D (not on
 *   user-supplied lattices).
 * ------------------------------------------------------------------------- */
typedef enum { MRTLB_NSE_INC = 0, MRTLB_NSE_COMP = 1, MRTLB_NCDE = 2, MRTLB_CDE = 3 } mrtlb_model;

typedef struct {
  int model;         /* mrtlb_model */
  double rho0;       /* NSE_INC reference density; deviation reference */
  double s0, s1, s_shear, s_bulk, s3, s_high;
  int m30;           /* NSE: include M30 = rho uuu */
  double D0, D2;     /* NCDE */
  double adv_u[3];   /* NCDE */
  /* Bounds the caller guarantees over the whole run, used only by
   * MRTLB_I16_DEV to size its fixed-point ranges: u_bound >= max |u|,
   * dev_bound >= max |rho - rho0| / rho0 (NSE) or max |phi| (NCDE).
   * Both 0 (the default) selects the uniform range |f_bar - w rho_ref| <= 2 w. */
  double u_bound, dev_bound;
  /* General NCDE (eq. M-NCDE-6): the auxiliary first moment gains
   * -S1 (A1 d_t B_bar + A2 div D_bar) with B_bar = phi b_bar and
   * D_bar = phi I, here gn_bt = A1 b_bar and gn_dd = diag(A2) per axis,
   * lagged like the rest of M1G (phi^n - phi^{n-1}; central difference of
   * phi^{n-1}).  Recovers phi_t + div(phi u) = div(D grad phi)
   * + dt sum_a gn_bt_a d_a d_t phi + dt sum_a gn_dd_a d_a^2 phi
   * (K1 = dt A1, K2 = dt A2).  NCDE only; zero otherwise.  The explicit
   * lagged d_t term limits |gn_bt| (order 1 is unstable). */
  double gn_bt[3], gn_dd[3];
  /* NCDE source S = src_q + src_k phi (F_j with M0F = S, M1F = 0, eqs.
   * M-NCDE-4, M-NCDE-5; |src_k| < 1) and the scheme of eq. (2-1):
   * three_level = 0: full correction (theta = gamma = 1, shifted f_bar,
   *   phi = sum f_bar + S/2 (eq. 2-4-1), solved for phi; the initial state
   *   is f_eq - w S/2);
   * three_level = 1: explicit three-level scheme (theta = 1, gamma = 0,
   *   unshifted f, phi = sum f, F + (F(t) - F(t - dt))/2 with F(t - dt)
   *   from the stored phi^{n-1}; initial state f_eq).
   * read_moments and conserved report phi of the chosen scheme.  The NSE
   * models take three_level too (see g_share below); src_q and src_k are
   * zero for every model but the NCDE. */
  double src_q, src_k;
  int three_level;
  /* NSE uniform mass source S (with g_share = 0: M0F = S, M1F = F,
   * M2F = 0, eq. M-NSEs-5 with S_G = 0): rho = sum f_bar + S/2 (eq. 2-4-2)
   * and M2G = (I - S2/2)[uF + Fu + (cs^2 I - uu) S] (eq. M2G-1 with
   * S_bar = S; for isothermal p, d_t p I + div(p u I) = cs^2 S I; eq.
   * M2Ga-1 for NSE_INC).  The initial state is f_eq - F/2.  A field S(x)
   * replaces it with mrtlb_set_mass_source_field.  Runs in the forced
   * kernel: the solve needs has_force (a zero force field is fine); EINVAL
   * otherwise and for the NCDE and CDE. */
  double mass_src;
  /* NSE partial correction (eqs. 2-4-0, 2-4-2, M-NSEs-2, M-NSEs-4-0): the
   * share g_share in [0, 1] of the body force and of the mass source that
   * the auxiliary distribution G carries, F_G = g F and S_G = g S (the rest,
   * F_F and S_F, is carried by the source distribution F), with
   *   rho = sum f + (lambda1 S_G + h S_F)/2,
   *   rho u = sum c f + (lambda2 F_G + h F_F)/2,
   *   M0G = (1 - s0 lambda1/2) S_G, M1G = (I - lambda2 S1/2) F_G,
   *   M2G = M2G_bar - lambda1 S20 S_G/2, S20 = cs^2 (s0 I - S2 I)
   * (the raw-moment block of the Hermite-space collision; S10 = S21 = 0),
   * h = 1 for the full correction and h = 0 for three_level = 1, which for
   * the NSE is the explicit three-level scheme of eq. (2-1) with theta = 1,
   * gamma = 0: unshifted f, F + (F(t) - F(t - dt))/2 with F(t - dt) the
   * force of the previous step (mrtlb_set_force_field), equal to the
   * current force on the first step after mrtlb_init_fields.  g = 0,
   * lambda1 = lambda2 = 1 is the full correction above; lambda1 = lambda2 = 1
   * gives the same scheme for every g.  The scheme is second order when
   * (1 - lambda1) S_G and (1 - lambda2) F_G do not vary in time and, for
   * the three-level scheme, div F_F = 0 (eq. M-NSEs-5).  The initial state
   * subtracts half a distribution of raw moments (lambda1 S_G + h S_F,
   * lambda2 F_G + h F_F, 0), so rho and u read back as given.  With
   * g_share = 0 (a zero-initialized descriptor) lambda1 and lambda2 act on
   * nothing.  Other models: g_share = 0 (EINVAL otherwise), lambdas ignored. */
  double g_share, lambda1, lambda2;
  /* NSE: the form of M2G_bar.  0: the local closed form above.  1: the
   * gradient form (eqs. M2G-1, M2G): NSE_COMP takes (d_t p + div(p u)) I,
   * p = cs^2 rho, in place of cs^2 S I; NSE_INC (rho = rho0, p = cs^2 rho_bar)
   * takes F_bar = F - cs^2 grad(rho_bar) and S_bar = S - d_t rho_bar in place
   * of F and S.  d_t is the backward difference of this step's value and the
   * previous step's, grad and div central differences (spacing c_a dt) of
   * the previous step's rho and rho u, which the solve keeps per node (two
   * slots of d + 1 values for NSE_COMP, 1 for NSE_INC, FP64 or FP32 as the
   * arithmetic).  The history before t = 0 follows the continuity equation:
   * rho^{-1} = rho^0 - dt (S - div(rho u)^0), (rho u)^{-1} = (rho u)^0.
   * One node per lane; storages FP64, FP32, FP32_DEV and FP32_DEV_F64;
   * compiled lattices; NSE_COMP on the multispeed lattices only (k = 0,
   * M30 = rho uuu).  EINVAL otherwise.  mrtlb_write_populations does not
   * set the history. */
  int m2g_form;
} mrtlb_model_desc;

/* Population storage in HBM (compute is FP64 for MRTLB_FP64 and
 * MRTLB_FP32_DEV_F64, FP32 otherwise):
 *   FP64      f_bar, double
 *   FP32      f_bar, float
 *   FP32_DEV  f_bar - w_j rho_ref, float
 *   FP32_DEV_F64  f_bar - w_j rho_ref, float (RNE from the FP64 result),
 *             with FP64 arithmetic: the bytes of FP32_DEV without the FP32
 *             rounding of every intermediate (the force field and the NCDE
 *             history are FP64)
 *   FP16_DEV  (f_bar - w_j rho_ref) * 128 / w_j, IEEE half (RNE)
 *   BF16_DEV  same, bfloat16 (RNE)
 *   I16_DEV   (f_bar - w_j rho_ref) * 32767 / (A_j w_j), int16 fixed point
 *             (RNE, saturating at +-A_j w_j).  A_j = 2 when u_bound and
 *             dev_bound are 0; otherwise, with t_j = |c_j| u_bound / cs^2,
 *             r = dev_bound and U = u_bound,
 *               A_j = 2 [r + (1 + r)(exp(t_j) - 1 + U^2 / (2 cs^2))],
 *             twice a bound on |f_eq,j - w_j rho_ref| / w_j (the equilibrium
 *             is a truncated series in c_j.u / cs^2 whose terms the exp
 *             series dominates); the factor 2 covers the non-equilibrium part.
 * rho_ref = rho0 (NSE) or 0 (NCDE).  Each FP32 value is rounded once to
 * the 16-bit format. */
typedef enum { MRTLB_FP64 = 0, MRTLB_FP32 = 1, MRTLB_FP32_DEV = 2, MRTLB_FP16_DEV = 3, MRTLB_BF16_DEV = 4,
               MRTLB_I16_DEV = 5, MRTLB_FP32_DEV_F64 = 6 } mrtlb_storage;

/* Create a solve on a periodic grid n[0] x n[1] (x n[2] in 3D; n[2] = 1 in
 * 2D).  Allocates two population buffers (pull streaming, double-buffered),
 * the force field and a mass-source field (d + 1 node fields) if has_force,
 * for the NCDE two phi history fields, for the NSE gradient form of
 * M2G_bar (m2g_form = 1) two slots of its history, and for a user-supplied
 * lattice (MRTLB_CUSTOM) the step kernel's table of its velocities (per
 * population: weight, storage scales, the monomials of e_j up to third
 * order, index and source-row offset; a few KB).
 * The lattice is copied; it may be destroyed afterwards.
 * Errors: EINVAL (sizes < 1, a size below the largest lattice offset, a
 * population buffer of 4 GiB or more, rates outside (0, 2), negative or
 * non-finite u_bound / dev_bound,
 * unknown model or storage, NSE_INC with rho0 <= 0), ENOMEM (footprint over
 * the remaining budget; nothing allocated), EDEVICE. */
mrtlb_status mrtlb_solve_create(mrtlb_ctx* ctx, const mrtlb_lattice* lat, const mrtlb_model_desc* model,
                                const int64_t n[3], int storage, int has_force, mrtlb_solve** out);
/* Device bytes mrtlb_solve_create would allocate.  model is the
 * mrtlb_model kind, plus MRTLB_FOOTPRINT_M2G_GRADIENT for m2g_form = 1. */
#define MRTLB_FOOTPRINT_M2G_GRADIENT 0x100
mrtlb_status mrtlb_solve_footprint(const mrtlb_lattice* lat, const int64_t n[3], int storage, int model,
                                   int has_force, size_t* bytes);
/* Bytes of one population buffer of a solve on this grid and storage.  The
 * buffer is row-blocked: for each grid row (y fastest, then z) its b
 * population rows back to back, each of pitch elements (nx rounded up to a
 * multiple of 32), x fastest; elements of the storage's type (8, 4 or 2
 * bytes, values as in mrtlb_storage).  f_bar_j of node (x, y, z) is the
 * element ((z' * ny + y') * b + j) * pitch + x' with (x', y', z') =
 * (x, y, z) - e_j modulo (nx, ny, nz): where the next step's pull gather
 * reads it. */
mrtlb_status mrtlb_population_bytes(const mrtlb_lattice* lat, const int64_t n[3], int storage, size_t* bytes);
/* As mrtlb_solve_create, but the two population buffers are the caller's:
 * f0 and f1 are device pointers on the context's device (for example two
 * torch tensors' data), each at least mrtlb_population_bytes long and
 * 16-byte aligned.  The solve reads and writes them in the layout above
 * (which of the two holds the current state alternates with the step
 * parity) and never frees them; the caller keeps them alive and unused by
 * other work until mrtlb_solve_destroy.  The remaining device memory
 * (parameters, force and history fields) is the library's and counts
 * against the budget.  Errors: as mrtlb_solve_create, and EINVAL for NULL,
 * equal, overlapping or misaligned buffers and for pointers that are not
 * device memory on the context's device. */
mrtlb_status mrtlb_solve_create_external(mrtlb_ctx* ctx, const mrtlb_lattice* lat, const mrtlb_model_desc* model,
                                         const int64_t n[3], int storage, int has_force, void* f0, void* f1,
                                         mrtlb_solve** out);
/* Destroy every solve before its context. */
void mrtlb_solve_destroy(mrtlb_solve* s);

/* Initial state: f_bar(x, 0) = f_eq(rho_or_phi, u) - F/2 (NSE) or
 * f_eq(phi) (NCDE).  rho_or_phi: N values (rho_bar for NSE_INC, rho for
 * NSE_COMP, phi for NCDE and CDE); u: d*N values (the velocity field for
 * the CDE; ignored for NCDE, may be NULL);
 * force: d*N values or NULL (required iff the solve has a force field).
 * Resets the step counter.  Synchronous. */
mrtlb_status mrtlb_init_fields(mrtlb_solve* s, const double* rho_or_phi, const double* u, const double* force);

/* How the step kernel evaluates the Hermite transforms (a solve setting):
 *   MRTLB_TRANSFORM_VALU  (default) structured monomial sums on the vector
 *                         ALUs, every lattice, storage and model;
 *   MRTLB_TRANSFORM_MFMA  dense products on the matrix cores: the forward
 *                         transform as the monomial matrix of order <= 3
 *                         (times each population's storage scale, f16 hi + lo)
 *                         against the stored int16 numbers (two exact f16
 *                         chunks each), the back-transform as its transpose
 *                         (times the output weights, bf16 hi + lo) against the
 *                         monomial coefficients (bf16 hi + lo), FP32
 *                         accumulation; the relaxation in between is the same
 *                         FP32 code.  3D lattices (|e| <= 2), MRTLB_I16_DEV
 *                         storage, NSE models without a force field, a row
 *                         pitch (nx rounded up to 32) that is a multiple of 64.
 * The stored format is the same for both, so a solve may switch at any step;
 * results agree to the int16 storage's precision, not bit for bit.
 * Errors: EINVAL (unknown transform, or MFMA outside the cases above),
 * ENOMEM (16 KB of tables beyond the budget), EDEVICE. */
typedef enum { MRTLB_TRANSFORM_VALU = 0, MRTLB_TRANSFORM_MFMA = 1 } mrtlb_transform;
mrtlb_status mrtlb_solve_set_transform(mrtlb_solve* s, int transform);

/* CDE only: replace the velocity field u(x) (d*N values, layout as in
 * mrtlb_init_fields) from the next step on, for a velocity that changes in
 * time, u(x, t): the steps use the field last set.  Waits for the work
 * enqueued before it.  Errors: EINVAL (NULL, not a CDE solve), ENUMERIC
 * (non-finite value), EDEVICE. */
mrtlb_status mrtlb_set_velocity_field(mrtlb_solve* s, const double* u);

/* NSE solves created with has_force: replace the body force F(x) (d*N
 * values, layout as in mrtlb_init_fields) from the next step on, for a force
 * that changes in time, F(x, t) (eq. 2-1 evaluates F at the step's time).
 * For the three-level scheme with g_share < 1 the next step adds
 * (1 - g_share)(F - F_prev)/2 to the first moment, F_prev being the force
 * of the previous step; the first such call allocates d*N reals (8 or 4
 * bytes, as the force field) for F_prev, kept until mrtlb_solve_destroy.
 * Waits for the work enqueued before it.  Errors: EINVAL (NULL, not an NSE
 * solve with a force field), ENUMERIC (non-finite value), ENOMEM, EDEVICE. */
mrtlb_status mrtlb_set_force_field(mrtlb_solve* s, const double* force);

/* NSE solves created with has_force: the mass source as a field S(x) (N
 * values, node order as rho in mrtlb_init_fields), in place of the uniform
 * mass_src, from the next step on (and for mrtlb_init_fields if set before
 * it); each step adds S(x) to the zeroth moment and rho = sum f + cS S(x)
 * as for the uniform source (eqs. M-NSEs-2, 2-4-2).  The three-level scheme
 * keeps the previous source as it keeps the previous force.  The field is
 * stored beside the force (the forced solve reserves d + 1 node fields).
 * Waits for the work enqueued before it.  Errors: EINVAL (NULL, not an NSE
 * solve with a force field), ENUMERIC (non-finite value), ENOMEM, EDEVICE. */
mrtlb_status mrtlb_set_mass_source_field(mrtlb_solve* s, const double* S);

/* Enqueue nsteps >= 0 collide-and-stream steps (asynchronous). */
mrtlb_status mrtlb_step(mrtlb_solve* s, int64_t nsteps);

/* Same, and return the device time of those steps in *ms, measured with HIP
 * events recorded on the context stream around the launches (synchronous). */
mrtlb_status mrtlb_step_timed(mrtlb_solve* s, int64_t nsteps, double* ms);

/* Streaming alone, a measurement aid: npasses >= 0 passes of the pull
 * streaming of eq. (2-2), f_j(x) <- f_j(x - e_j) on the periodic grid, with
 * no collision; every stored number moves unchanged.  Each pass runs the
 * step kernel's tiles, gather, tile order and store policy with nothing
 * between load and store, so its rate bounds the step kernel's on the same
 * solve.  The step counter, drift reference, force and M2G history are left
 * as they were: the populations afterwards are not a state of the method's
 * time stepping.  If ms is not NULL the call returns the device time of the
 * passes in *ms (HIP events on the context stream, synchronous); otherwise
 * it is asynchronous.  Errors: EINVAL (NULL solve, npasses < 0, a
 * user-supplied lattice), EDEVICE. */
mrtlb_status mrtlb_stream_only(mrtlb_solve* s, int64_t npasses, double* ms);

/* The launch shape chosen for a solve's step kernel, a measurement aid (the
 * choices are measured heuristics of the library; the environment variables
 * MRTLB_STEP_VEC, MRTLB_XCD_ORDER and MRTLB_STEP_WG_PER_CU, read when the
 * solve is created, override them for tuning runs).  *nodes_per_lane:
 * consecutive x-nodes per thread (1, 2 or 4); *xcd_ranges: 1 if the tiles
 * run in contiguous ranges per XCD, 0 if in dispatch order; *wg_per_cu: the
 * workgroups per compute unit that the occupancy cap allows (LDS reserved
 * and not used), 0 if uncapped; *workgroups: workgroups of one step launch.
 * Any output pointer may be NULL.  A batched launch over several solves
 * takes its own tile order and cap from the whole batch.  Errors: EINVAL
 * (NULL solve).  No device work. */
mrtlb_status mrtlb_solve_launch_shape(const mrtlb_solve* s, int* nodes_per_lane, int* xcd_ranges, int* wg_per_cu,
                                      int64_t* workgroups);

/* Drift correction of the conserved totals.  The collision conserves mass,
 * and momentum without a force, exactly (Sec. II, eq. M-NSEs-1); the
 * rounding of the stored populations does not.  With every > 0, after each
 * `every` steps of mrtlb_step / mrtlb_batch_step the library takes the FP64
 * totals of the populations (mass: rho_bar, rho or phi; momentum for the NSE
 * models without a force) and adds their difference to the totals recorded
 * at the reference point, spread evenly over the nodes, to the zeroth and
 * first moments of the next step's collision.  The reference point is the
 * latest of mrtlb_init_fields, mrtlb_write_populations and this call.  Each
 * check costs one FP64 reduction pass over the populations and a host
 * synchronisation.  every = 0 (the default) turns it off.
 * Errors: EINVAL (NULL solve, every < 0, a CDE solve: its total changes),
 * EDEVICE, ENUMERIC (non-finite state at the reference point). */
mrtlb_status mrtlb_set_drift_correction(mrtlb_solve* s, int64_t every);

/* Advance solve i of the array by nsteps[i] >= 0 steps.  Solves that share
 * lattice, model, storage and force go into one kernel launch per step (the
 * ones that have finished drop out of later launches); groups run one after
 * the other on the context stream.  Solves must belong to the same context
 * and appear once.  Each solve's result equals mrtlb_step on it alone, bit
 * for bit.  Synchronous (returns when the steps have run). */
mrtlb_status mrtlb_batch_step(mrtlb_solve* const* solves, int n, const int64_t* nsteps);

/* rho_or_phi (N) and u (d*N, may be NULL) at the current time, eq. (2-4-2)
 * / (2-4-1): rho_bar = sum f_bar, u = (sum c f_bar + F/2)/rho_m; NCDE
 * phi = sum f_bar + S/2 (full correction) or sum f (three-level scheme).
 * Synchronous. */
mrtlb_status mrtlb_read_moments(mrtlb_solve* s, double* rho_or_phi, double* u);

/* Domain totals in FP64 with a fixed reduction order: mass = sum rho_bar
 * (or sum phi, phi as read_moments gives it), momentum[d] =
 * sum (sum c f_bar + F/2).  Returns ENUMERIC if a
 * stored value is not finite.  Synchronous. */
mrtlb_status mrtlb_conserved(mrtlb_solve* s, double* mass, double* momentum);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * totals as mrtlb_conserved, bit for bit, computed without any device or
 * host allocation.  The FP64 partial sums live in a scratch array of the
 * library, 4 MiB per GPU, held from the first context on that GPU until the
 * process ends and shared by every call on that GPU: calls that overlap on
 * one GPU (several threads, or contexts on different streams) race, and
 * each call overwrites what the previous one left.  The solve's sums need
 * (b + force components) * (ceil(N / 4096) + 1) doubles, e.g. 1.7 MB for
 * rD3Q53 at 256^3; larger solves get EINVAL (use mrtlb_conserved).  Errors
 * otherwise as mrtlb_conserved.  Synchronous. */
mrtlb_status mrtlb_conserved_noalloc(mrtlb_solve* s, double* mass, double* momentum);

/* Checkpoint / restore of f_bar at the current time (b*N values). */
mrtlb_status mrtlb_read_populations(mrtlb_solve* s, double* f);
mrtlb_status mrtlb_write_populations(mrtlb_solve* s, const double* f);

/* Steps taken since the last init (or write_populations keeps the count). */
int64_t mrtlb_solve_steps(const mrtlb_solve* s);

#ifdef __cplusplus
}
#endif
#endif /* MRTLB_H */
