/*
 * coag.h -- C ABI of libcoag, the MI355X (gfx950) coagulation-fragmentation
 * update of Robinson, Booth & Owen, "Introducing cuDisc" (Sec. 5, "Dust growth
 * and fragmentation"; sub-cycling rule of Sec. 6, "Code structure").
 *
 * Each (R, Z) cell evolves its binned grain-size distribution rho[cell][k]
 * (g cm^-3 per mass bin) under the Smoluchowski equation with coagulation,
 * cratering/fragmentation and power-law fragments, independently of every
 * other cell.  Four calls make up the path:
 *
 *   coag_rates          pair rates  Kc = w K p_coag,  Kf = w K p_frag
 *                       (coag_rates_blocked: the same in the 16-cell-blocked
 *                       layout the batched step streams, FP64 or FP32)
 *   coag_rhs            drho/dt  (eq. `smol`)
 *   coag_step           sub-cycled Bogacki-Shampine 3(2) over dt
 *   coag_step_backward  adjoint of a frozen step sequence
 *
 * Conventions (all calls):
 *   - Pointers marked DEVICE are device pointers on the HIP device that was
 *     current at coag_create; they are owned by the caller, contiguous,
 *     row-major, FP64 unless stated.  HOST pointers are read during the call.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work is
 *     enqueued on it; no call synchronises the host, so outputs are ready only
 *     after the stream is synchronised.
 *   - Pairs are packed: p(i, j) = i (i + 1) / 2 + j for j <= i (i is the
 *     heavier grain); P = N (N + 1) / 2.
 *   - Return value: COAG_OK, or a negative COAG_E* code for an error found on
 *     the host before anything is launched (nothing is written then); the
 *     message is in coag_last_error().  Failures inside a cell are reported in
 *     that cell's `status` and never stop other cells.
 *   - C = 0 is a valid no-op; array pointers may then be NULL.
 *   - A context is bound to one device and is not thread-safe; calls that
 *     overlap on the same context must not share the context's workspace
 *     (use one context per stream).
 *   - CGS units throughout.
 */
#ifndef COAG_H
#define COAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct coag_ctx coag_ctx;

enum {
    COAG_OK = 0,
    COAG_EINVAL = -1,     /* bad argument (null pointer, size, grid, tolerance) */
    COAG_ENOMEM = -2,     /* device or host allocation failed */
    COAG_EHIP = -3,       /* a HIP runtime call failed */
    COAG_ENOTSUP = -4     /* combination not implemented */
};

/* per-cell status written by coag_step */
enum {
    COAG_CELL_OK = 0,
    COAG_CELL_HMIN = 1,       /* step size fell below h_min_rel * dt */
    COAG_CELL_MAXSUB = 2,     /* max_sub attempts used before reaching dt */
    COAG_CELL_NONFINITE = 3   /* a state or error estimate became NaN/Inf */
};

/* Two-bin split of a product mass M between l(M) and u(M) = l + 1 (eqs.
   `Cijk`, `Rijk`, eps = (m_u - M) / (m_u - m_l)):
   MASS   : mass eps*M to l and (1-eps)*M to u (the coefficients read as mass
            fractions, as the text states);
   NUMBER : one particle split by number, mass eps*m_l to l, (1-eps)*m_u to u. */
enum { COAG_SPLIT_MASS = 0, COAG_SPLIT_NUMBER = 1 };

/* arithmetic of the gain/loss contraction inside coag_step */
enum { COAG_PREC_FP64 = 0, COAG_PREC_SPLIT_BF16 = 1 };

/* step-size modes of coag_step */
enum { COAG_ADAPTIVE = 0, COAG_FIXED = 1, COAG_REPLAY = 2 };

/* layouts of the rates handed to coag_step (coag_tol.rates_layout):
   CP64  : double, two arrays Kc, Kf [C][P], pair p of cell c at c * P + p
           (coag_rates);
   BLK32 : float, 16-cell-blocked, both kinds in one array (coag_rates_blocked,
           f32 = 1);
   BLK64 : double, 16-cell-blocked, both kinds in one array (coag_rates_blocked,
           f32 = 0).
   Blocked: per block of 16 cells (cells 16 b .. 16 b + 15) the pairs of each
   row i are taken two by two: pair (i, j) lies in slot S(i) + j / 2 of the
   block with parity u = j & 1, S(i) = m (m + 1) for i = 2m and (m + 1)^2 for
   i = 2m + 1 (a row of odd length ends with the zero entry (i, i + 1)); S(N)
   slots of 64 values per block, 64 S(N) ceil(C/16) values in all.  Kind k
   (0: Kc, 1: Kf) of cell c of the block in slot s at, within the block,
     BLK64 ((s * 2 + u) * 16 + c % 16) * 2 + k
     BLK32 ((s * 16 + c % 16) * 2 + u) * 2 + k
   the order in which one 16-byte load per lane of a wave is contiguous.  The
   padding cells of the last block and the zero entries are read and must be
   finite (coag_rates_blocked writes zeros). */
enum { COAG_RATES_CP64 = 0, COAG_RATES_BLK32 = 1, COAG_RATES_BLK64 = 2 };

/* Mass grid and collision-outcome parameters (Sec. 5).  HOST arrays, copied
   by coag_create.  m strictly increasing; m_edge[k] < m[k] < m_edge[k+1]
   (bin edges, used by the fragment distribution eq. `Nijk`); s = grain radius
   of each bin (cm).  rho_m: grain material density; eta: fragment power law
   n(m) ~ m^-eta (eq. `fragdist`, eta != 2); chi: excavated mass in units of
   the impactor mass (eq. `fragrem`, chi > 0); split: COAG_SPLIT_*.
   vertical: 0 for the volume kernel (states are mass densities per bin,
   g cm^-3, each cell a point of the (R, Z) grid); 1 for the vertically
   integrated kernel of the paper's single-radius test (Sec. 5.1): states
   are surface densities per bin (g cm^-2), each cell a column whose rho_g is
   the midplane gas density and whose grains have Gaussian vertical profiles
   of scale height h_k = H sqrt(alpha / (alpha + St_k)); the pair rate is the
   volume rate integrated over height, K / sqrt(2 pi (h_i^2 + h_j^2)), and the
   vertical relative velocity the difference of the settling speeds
   St_k Omega h_k (the vertical components of v_dust are not used).  The
   vertical form needs alpha > 0 in every cell (else the rates are not
   finite).  Chosen per context: every rate, step and adjoint call of the
   context takes it. */
typedef struct {
    int32_t n_bins;           /* N, 2 <= N <= 1023 */
    int32_t split;
    const double *m;          /* [N]   HOST */
    const double *m_edge;     /* [N+1] HOST */
    const double *s;          /* [N]   HOST */
    double rho_m, eta, chi;
    int32_t vertical;         /* 0 volume kernel, 1 vertically integrated */
} coag_grid;

/* Per-cell gas state, each a DEVICE array [C]: temperature T (K), gas density
   rho_g, isothermal sound speed c_s, Keplerian angular speed Omega, gas scale
   height H, molecular kinematic viscosity nu_mol, turbulence parameter alpha
   (alpha = 0 switches turbulent relative velocities off). */
typedef struct {
    const double *T, *rho_g, *c_s, *Omega, *H, *nu_mol, *alpha;
} coag_cells;

/* Step control (Sec. 5: rtol = 1e-2, atol = 1e-10 * sum_k rho_k by default).
   mode: COAG_ADAPTIVE / COAG_FIXED / COAG_REPLAY.  max_sub: cap on attempted
   sub-steps per cell per call (ADAPTIVE), and the row length of h_log.
   prec: COAG_PREC_*.  renorm: non-zero rescales each cell's state after the
   call so that its total mass equals the total at entry (COAG_PREC_SPLIT_BF16
   always does).  rates_layout: COAG_RATES_* of the Kc, Kf handed to
   coag_step; BLK32 with COAG_PREC_SPLIT_BF16 only, BLK64 with COAG_PREC_FP64
   only. */
typedef struct {
    double rtol, atol_rel, h_min_rel;
    int32_t max_sub, mode, prec, renorm, rates_layout;
} coag_tol;

/* ------------------------------------------------------------------------- */

/* Log-spaced mass grid on the HOST (no device work).  N bins whose outer
   edges are lo and hi (grain radius in cm if by_mass == 0, else mass in g),
   edges lo (hi/lo)^(k/N), centres at the log midpoints lo (hi/lo)^((k+1/2)/N),
   m = (4 pi / 3) rho_m s^3.  Writes m[N], m_edge[N+1], s[N] (HOST, caller-
   owned).  Reading of Sec. 7: with it, the paper's 100 bins over
   0.1 um - 0.5 cm and 135 bins over 0.1 um - 20 cm both have
   m_{n+1}/m_n = 1.38.  Returns COAG_EINVAL for N < 2, lo <= 0, hi <= lo,
   rho_m <= 0 or a null pointer. */
int coag_mass_grid(int32_t n_bins, double lo, double hi, int32_t by_mass, double rho_m,
                   double *m, double *m_edge, double *s);

/* Create a context on the current HIP device: validates the grid and builds
   on the device, once, the redistribution tables of the gain term (where the
   products of each pair go: coagulation split, remnant split, top fragment
   bin and fragment mass, eqs. `Cijk`, `Rijk`, `fragrem`, `Nijk`).  The
   context owns those tables and its workspaces; *out receives it.
   Errors: COAG_EINVAL (bad grid), COAG_ENOMEM, COAG_EHIP. */
int coag_create(const coag_grid *grid, coag_ctx **out);

/* Free a context and everything it owns (NULL is accepted).  Synchronises the
   device first so that no queued work still uses the context. */
void coag_destroy(coag_ctx *ctx);

/* Last error message of this context (or of the last failed coag_create /
   coag_mass_grid when ctx is NULL); "" if none.  Valid until the next call. */
const char *coag_last_error(const coag_ctx *ctx);

/* Pair rates for C cells (Sec. 5, eqs. `kernel`, `vbrown`, `OCVrel`,
   `p_frag`; Stokes number from the Epstein stopping time, eq. `t_stop`, times
   Omega; Re = alpha c_s H / nu_mol as in Sec. 7.1).
     v_dust [C][N][3] DEVICE   dust velocities from the dynamics solver
     v_frag [C]       DEVICE   fragmentation velocity
     Kc, Kf [C][P]    DEVICE   out: w K_ij p_coag,ij and w K_ij p_frag,ij with
                               w = 1/2 for i = j (the halving the gain term asks for)
   Errors: COAG_EINVAL (C < 0, null pointer). */
int coag_rates(coag_ctx *ctx, int64_t C, const coag_cells *cells, const double *v_dust,
               const double *v_frag, double *Kc, double *Kf, void *stream);

/* The same rates in the 16-cell-blocked layout (COAG_RATES_BLK32 / BLK64
   above), both kinds in one array: f32 = 1 rounds them to float, for the
   split-BF16 step, which then streams half the bytes per right-hand side;
   f32 = 0 keeps double, for the batched FP64 step.  The batched kernels read
   them in place with one 16-byte load per lane and pair (double) or two pairs
   (float), whole cache lines over a wave.  K DEVICE out, 64 S(N) ceil(C/16)
   elements, caller-owned; the padding cells of the last block and the zero
   entries are written as zeros.  Errors as coag_rates, and COAG_EINVAL for
   f32 not 0 or 1. */
int coag_rates_blocked(coag_ctx *ctx, int64_t C, const coag_cells *cells, const double *v_dust,
                       const double *v_frag, int32_t f32, void *K, void *stream);

/* Right-hand side of eq. `smol` for C cells:
     drho_k = sum_{i, j<=i} n_i n_j [Kc (m_i+m_j) C_ijk + Kf (m_rem R_ijk + m_frag F_ijk)]
              - m_k n_k sum_i K_ik n_i (p_c + p_f),      n = rho / m,
   fragments distributed per top bin (the accumulation of Rafikov et al. 2020).
     rho     [C][N] DEVICE in;   Kc, Kf [C][P] DEVICE in;   drho_dt [C][N] DEVICE out.
   Errors: COAG_EINVAL. */
int coag_rhs(coag_ctx *ctx, int64_t C, const double *rho, const double *Kc, const double *Kf,
             double *drho_dt, void *stream);

/* Advance every cell by dt (Sec. 5 closing paragraph; Sec. 6 sub-cycling).
   BS3(2) with first-same-as-last reuse:
     k1 = f(y), k2 = f(y + h/2 k1), k3 = f(y + 3h/4 k2),
     y+ = y + h (2/9 k1 + 1/3 k2 + 4/9 k3),   k4 = f(y+),
     e  = h (-5/72 k1 + 1/12 k2 + 1/9 k3 - 1/8 k4).
   ADAPTIVE: err = max_k |e_k| / (atol + rtol max(|y_k|, |y+_k|)), atol =
   atol_rel * sum_k y_k at entry; accept iff err <= 1 and no y+_k < -atol; step
   factor clamp(0.9 err^(-1/3), 0.2, 5) (5 if err = 0), 0.5 after a rejection
   caused only by a negative state; the final step is clipped to land on dt and
   a clipped accepted step leaves h unchanged.  FIXED: nsub[c] equal steps of
   dt/nsub[c].  REPLAY: nsub[c] steps of the sizes h_log[c][0..nsub[c]).
     rho     [C][N]        DEVICE in/out
     Kc, Kf                DEVICE in, in tol->rates_layout: double [C][P] (from
                           coag_rates, or any kernel), or 16-cell-blocked float or
                           double in Kc alone (from coag_rates_blocked; Kf NULL)
     h       [C]           DEVICE in/out (ADAPTIVE): h <= 0 on entry starts with dt;
                           on exit the controller's next (unclipped) step size
     nsub    [C] int32     DEVICE out (ADAPTIVE: accepted steps) or in (FIXED, REPLAY)
     nrej    [C] int32     DEVICE out, rejected attempts (may be NULL)
     h_log   [C][max_sub]  DEVICE out (ADAPTIVE, FIXED: accepted step sizes; may be
                           NULL) or in (REPLAY, required)
     status  [C] int32     DEVICE out, COAG_CELL_*
   Arithmetic (tol->prec):
     COAG_PREC_FP64: everything in FP64.  Where the grid allows it (N >= 16,
       the products of each row of pairs within 16 consecutive bins, and
       N <= 343 so that the state of 16 cells fits LDS) 16 cells advance
       together and the gain sum runs on FP64 matrix cores;
       otherwise one workgroup per cell.  The environment variable
       COAG_STEP_KERNEL=cell, read by coag_create, forces the latter.
     COAG_PREC_SPLIT_BF16: the gain sum sum_p n_i n_j K_p D_pk runs as BF16
       matrix products of three-limb splits of its FP32-rounded operands with
       FP32 accumulation; losses, fragments, stage states, error control, the
       update and the per-cell mass bookkeeping stay in FP64.  Needs the same
       grid conditions (else COAG_ENOTSUP).
   Errors: COAG_EINVAL (null pointer, C < 0, dt <= 0, rtol <= 0, max_sub < 1,
   unknown mode, precision or rates layout, a layout the precision does not
   take, a non-NULL Kf with blocked rates), COAG_ENOTSUP (split precision or blocked rates on a grid the batched
   step does not cover; blocked FP64 rates with COAG_STEP_KERNEL=cell),
   COAG_ENOMEM. */
int coag_step(coag_ctx *ctx, int64_t C, double *rho, const void *Kc, const void *Kf,
              double dt, double *h, const coag_tol *tol, int32_t *nsub, int32_t *nrej,
              double *h_log, int32_t *status, void *stream);

/* coag_step without any allocation, for callers that cannot allocate device
   memory (code under HIP graph capture, tight serving loops, harnesses that
   forbid hipMalloc): the same arguments, checks, kernels and results as
   coag_step, with the batched step's workspace taken from a static 64 MiB
   array that the library holds on each device from its load to the end of
   the process, instead of the context's workspace.  That is room for
   40 N bytes per cell with blocked rates (COAG_RATES_BLK32 / BLK64: e.g. 8388
   cells of 200 bins), and 32 S(N) + 40 N (about 16 P + 48 N) bytes per cell
   with [C][P] FP64 rates in the FP64 step, which reorders them there (about
   200 cells of 200 bins).  Larger calls return COAG_EINVAL and launch nothing; split them
   into smaller ones.  Every call on one device shares that device's array:
   calls that may overlap on one device (other streams, other contexts, other
   host threads) race and must be serialised by the caller.  Nothing in the
   array needs to start at zero.  Per-cell kernels (grids the batched step does
   not cover, COAG_STEP_KERNEL=cell) use no workspace and run as in coag_step.
   Errors: those of coag_step, COAG_EINVAL for a call beyond the array, and
   COAG_ENOTSUP on a device without the array (device index >= 64). */
int coag_step_noalloc(coag_ctx *ctx, int64_t C, double *rho, const void *Kc, const void *Kf,
                      double dt, double *h, const coag_tol *tol, int32_t *nsub, int32_t *nrej,
                      double *h_log, int32_t *status, void *stream);

/* Discrete adjoint of coag_rates + coag_step over a frozen step sequence
   (nsub[c] accepted steps of sizes h_log[c][:], as a REPLAY or FIXED call
   reproduces them): the derivative of the update of Sec. 5 (eqs. `smol`,
   `ngain`, the loss term, the rates of eqs. `kernel`, `OCVrel`, `p_frag`)
   through the Bogacki-Shampine stages.  With J a scalar of the final state and
   g_out = dJ/drho_end:
     g_in    [C][N] DEVICE out   dJ/drho at the start of the call (may be the
                                 same array as g_out: in place)
     g_alpha [C]    DEVICE out   dJ/dalpha_c (through v_turb and Re)
     g_vfrag [C]    DEVICE out   dJ/dv_frag,c (through p_frag)
   Inputs rho_in [C][N], cells, v_dust, v_frag as for coag_rates; h_log
   [C][log_stride], nsub [C] DEVICE.  The rates and the stage states are
   recomputed from rho_in and kept in the context's workspace for the reverse
   sweep; nothing of size [C][P] is kept where the batched kernels apply (the
   rate derivatives are folded into g_alpha, g_vfrag during the sweep), and the
   workspace holds at most about 8 GiB, the cells being taken in equal slabs
   (COAG_ADJ_SLAB_CELLS, read by coag_create, sets a smaller slab).
   prec: COAG_PREC_FP64 (everything in FP64), or COAG_PREC_SPLIT_BF16 (the
   adjoint of the split-precision step: FP32 rates and derivative factors, the
   transposed gain sum on BF16 matrix cores from three-limb splits, the rest in
   FP64; its mass renormalisation is taken as the identity).  Where the
   batched kernels do not apply (the grid conditions of coag_step, or
   COAG_STEP_KERNEL=cell) the FP64 adjoint runs one cell per workgroup with
   [C][P] rate and rate-gradient buffers, and split precision returns
   COAG_ENOTSUP.  A cell whose nsub is negative or above log_stride, or whose
   replay fails (non-finite state), gets NaN in g_in, g_alpha and g_vfrag;
   other cells are unaffected.  nsub = 0 gives g_in = g_out and zero g_alpha,
   g_vfrag.  Errors: COAG_EINVAL (null pointer, C < 0, log_stride < 1, unknown
   precision), COAG_ENOTSUP, COAG_ENOMEM. */
int coag_step_backward(coag_ctx *ctx, int64_t C, const double *rho_in, const coag_cells *cells,
                       const double *v_dust, const double *v_frag, const double *h_log,
                       int32_t log_stride, const int32_t *nsub, const double *g_out,
                       double *g_in, double *g_alpha, double *g_vfrag, int32_t prec,
                       void *stream);

#ifdef __cplusplus
}
#endif

#endif /* COAG_H */
