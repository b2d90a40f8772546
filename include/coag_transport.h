/* coag_transport.h -- C ABI of the dust transport step and of the scheduler
 * that couples it to the coagulation update (libcoag.so).
 *
 * Robinson, Booth & Owen, "Introducing cuDisc" (arXiv 2402.18471):
 *   Sec. 3, dynamics solver: each dust species a pressureless fluid with
 *     conserved Q = (rho, rho v_R, rho v_phi R, rho v_Z) (eq. `quants`),
 *     advective and diffusive fluxes (eqs. `dynfluxes`, `diffflux`,
 *     `Fdiffmom`), curvature and gravity sources and Epstein drag (eqs.
 *     `sources`, `dragforce`, `t_stop`), solved by the two-stage Godunov step
 *     listed after eq. `t_stop` with the Roe-averaged upwind flux of eqs.
 *     `roeav`, `riemann`; time step from the CFL rule (eqs. `dtCFL`,
 *     `dt_adv`, `dt_diff`).
 *   Sec. 6, code structure: the global step is the transport's CFL step, and
 *     the coagulation update runs, sub-cycling on its own, whenever the
 *     global time since its last call reaches the last sub-step it took.
 *
 * Grid (the poloidal grid of Sec. 7): n_r x n_z cells bounded by cylinders
 * R = R_edge[i] and cones Z = t_edge[j] R, cell c = i * n_z + j, t_edge[0] = 0
 * the midplane.  Cell volume (2 pi / 3)(R+^3 - R-^3)(t+ - t-); cylinder face
 * area 2 pi R^2 (t+ - t-); cone face area pi (R+^2 - R-^2) sqrt(1 + t^2) with
 * unit normal (-t, 1) / sqrt(1 + t^2); cell centre R_c = sqrt(R- R+),
 * Z_c = R_c (t- + t+) / 2.  Boundaries: zero-gradient at both radial edges
 * and the top, mirror (v_Z reversed) at the midplane.
 *
 * State: rho [C][N] (mass density per species, the same array the
 * coagulation calls take) and v [C][N][3] (v_R, v_phi, v_Z: the azimuthal
 * component absolute, not relative to Keplerian; the collision kernel only
 * uses velocity differences, so the same array serves as its v_dust), both
 * DEVICE, FP64.  Gas: the coag_cells arrays rho_g, c_s, H, alpha (viscosity
 * nu = alpha c_s H, the alpha prescription of Sec. 7) and v_gas [C][3].
 *
 * Errors are COAG_* codes of coag.h; the message is in
 * coag_transport_last_error.  Calls on one context are not thread-safe.
 */
#ifndef COAG_TRANSPORT_H
#define COAG_TRANSPORT_H

#include <stdint.h>

#include "coag.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct coag_tctx coag_tctx;

/* n_r >= 1, n_z >= 1; R_edge HOST [n_r + 1] increasing and > 0; t_edge HOST
   [n_z + 1] increasing with t_edge[0] = 0; GM = G M_* (cgs); Sc > 0 the
   Schmidt number (1 in the paper's runs); c_adv, c_diff the Courant numbers
   of eqs. `dt_adv`, `dt_diff` (0.4 and 0.2 by default); eps_floor >= 0 the
   dust-to-gas floor of each species (Secs. 2 and 7 speak of floor values
   without giving them): a species whose density in a cell ends either stage
   of a step below eps_floor rho_g takes the gas velocity there, its density
   kept; 0 = no floor. */
typedef struct {
    int32_t n_r, n_z;
    const double *R_edge;
    const double *t_edge;
    double GM, Sc, c_adv, c_diff;
    double eps_floor;
} coag_tgrid;

/* Create a transport context on the current device for N species of grain
   radii s (HOST [N], cm) and material density rho_m: the grid's geometry
   tables, the half-step workspace (4 C N doubles) and the gas tables each
   step refreshes (about 4 C doubles).  Errors: COAG_EINVAL, COAG_ENOMEM,
   COAG_EHIP. */
int coag_transport_create(const coag_tgrid *grid, int32_t N, const double *s, double rho_m,
                          coag_tctx **out);

/* Free a context (NULL accepted); synchronises the device first. */
void coag_transport_destroy(coag_tctx *t);

/* Last error message of the context, or of the last failed create when t is
   NULL; "" if none. */
const char *coag_transport_last_error(const coag_tctx *t);

/* CFL time step (eqs. `dtCFL`, `dt_adv`, `dt_diff`): the minimum over cells and
   species of c_adv min(dR / |v_R|, dZ / |v_Z|) and c_diff min(dR^2, dZ^2) /
   (nu / Sc), dR the cell's radial width, dZ its height at R_c; components and
   viscosities that are zero impose no limit (+inf if nothing does).  v DEVICE
   [C][N][3]; *dt_out HOST, written after the stream has finished the
   reduction (the call synchronises the stream). */
int coag_transport_dt(coag_tctx *t, const coag_cells *cells, const double *v, double *dt_out,
                      void *stream);

/* One transport step of dt (> 0) in place on rho [C][N] and v [C][N][3]
   (DEVICE): first-order fluxes at t^n, half update, half source and drag;
   second-order (piecewise-linear, van Leer-limited) fluxes at t^{n+1/2}, full
   update from t^n, full source and drag.  v_gas DEVICE [C][3].  Asynchronous
   on stream.  Empty cells (rho <= 0) get velocity 0. */
int coag_transport_step(coag_tctx *t, const coag_cells *cells, const double *v_gas, double *rho,
                        double *v, double dt, void *stream);

/* Scheduler statistics of one coag_evolve call. */
typedef struct {
    int64_t transport_steps;      /* CFL steps taken */
    int64_t coag_calls;           /* coagulation updates triggered */
    double t_reached;             /* global time at return */
    int32_t cells_failed;         /* cells with a non-zero coagulation status in the last call */
} coag_evolve_stats;

/* Evolve the disc over t_end (> 0) of global time (Sec. 6): repeat { dt = the
   CFL step, clipped to what remains; transport step; advance the clock; if the
   time since the last coagulation update reaches the trigger, or t_end is
   reached, run one coagulation update over that time (rates from the current
   velocities, then an ADAPTIVE coag_step under tol, h carried in h) and set
   the trigger to the smallest last sub-step h of the
   cells }.  The first trigger is the smallest h on entry (0: the first step
   triggers).  ctx: a coagulation context with the same N and grain radii,
   for the volume kernel (a vertically integrated one: COAG_EINVAL);
   v_frag DEVICE [C]; h DEVICE [C] in/out; tol: mode must be COAG_ADAPTIVE,
   prec COAG_PREC_FP64 or COAG_PREC_SPLIT_BF16 (rates in the matching blocked
   layout where the batched step applies to the context's grid; elsewhere
   FP64 runs the per-cell step on [C][P] rates, and split precision returns
   COAG_ENOTSUP before any work); max_steps caps the transport steps
   (COAG_EINVAL past it, state as reached).  Synchronises the stream once per transport step (to read dt).
   stats may be NULL. */
int coag_evolve(coag_ctx *ctx, coag_tctx *t, int64_t C, const coag_cells *cells,
                const double *v_gas, const double *v_frag, double *rho, double *v, double *h,
                double t_end, int64_t max_steps, const coag_tol *tol, coag_evolve_stats *stats,
                void *stream);

#ifdef __cplusplus
}
#endif

#endif /* COAG_TRANSPORT_H */
