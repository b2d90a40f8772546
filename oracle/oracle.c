/*
 * oracle.c -- plain FP64 CPU oracle of the coagulation-fragmentation update
 * (Robinson, Booth & Owen, "Introducing cuDisc", Sec. 5 "Dust growth and
 * fragmentation", and the sub-cycling rule of Sec. 6 "Code structure").
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the GPU
 * library; the two meet only through seeded inputs made elsewhere.
 *
 * Straight loops, FP64, no fast-math, no blocking or fusion beyond what the
 * equations state; OpenMP only over independent cells.
 *
 * Pins (tests/test_oracle_*.py): constant-kernel total number and second moment
 * against their closed forms and their exact BS3 recursions, additive-kernel
 * moments, exact mass conservation of every redistribution row, brute-force
 * discrete Smoluchowski on a linear grid, the Rafikov accumulation against the
 * dense per-pair fragment matrix, Ormel & Cuzzi asymptotes, the textbook
 * Brownian kernel, p_frag special values, and the hand adjoint against complex
 * step and central differences.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle_core.h"

/* ----- real instantiation of the forward arithmetic ---------------------- */
#define SC double
#define FN(name) r_##name
#define RE(x) (x)
#define SQRTT(x) sqrt(x)
#define EXPT(x) exp(x)
#include "oracle_fwd.inc"
#undef SC
#undef FN
#undef RE
#undef SQRTT
#undef EXPT

/* ------------------------------------------------------------------------- */
/* Mass grid (Sec. 7: log-spaced bins with a fixed ratio m_{n+1}/m_n).       */
/* The quoted size range is taken as the outer bin edges: N bins log-spaced  */
/* in radius (by_mass = 0, lo/hi in cm) or in mass (by_mass = 1, lo/hi in g) */
/* with edges x_k = lo (hi/lo)^(k/N), k = 0..N, and centres at the log       */
/* midpoints x_k = lo (hi/lo)^((k+1/2)/N).  With this reading the paper's    */
/* 100 bins over 0.1 um - 0.5 cm and 135 bins over 0.1 um - 20 cm both give  */
/* m_{n+1}/m_n = 1.38.  Masses m = (4 pi / 3) rho_m s^3.                     */
/* ------------------------------------------------------------------------- */
static double grid_mass(double x, int by_mass, double rho_m)
{
    return by_mass ? x : 4.0 * M_PI / 3.0 * rho_m * x * x * x;
}

int oracle_mass_grid(int N, double lo, double hi, int by_mass, double rho_m,
                     double *m, double *m_edge, double *s)
{
    if (N < 2 || !(lo > 0) || !(hi > lo) || !(rho_m > 0)) return -1;
    for (int k = 0; k <= N; ++k)
        m_edge[k] = grid_mass(lo * pow(hi / lo, (double)k / (double)N), by_mass, rho_m);
    for (int k = 0; k < N; ++k) {
        double x = lo * pow(hi / lo, (k + 0.5) / (double)N);
        m[k] = grid_mass(x, by_mass, rho_m);
        s[k] = by_mass ? cbrt(3.0 * x / (4.0 * M_PI * rho_m)) : x;
    }
    return 0;
}

/* Two-bin split of a product of mass M (eqs. `Cijk`, `Rijk`).
   l(M) = largest k with m_k <= M (an exact hit goes wholly to that bin),
   u = l + 1, eps = (m_u - M) / (m_u - m_l), 1 - eps = (M - m_l) / (m_u - m_l).
   MASS  : mass eps*M to l and (1-eps)*M to u   (C_ijk as a mass fraction)
   NUMBER: mass eps*m_l to l and (1-eps)*m_u to u (one particle split by number)
   Products at or above the top bin go wholly to N-1, below bin 0 wholly to 0. */
static void split_mass(const double *m, int N, double M, int split,
                       int *k, double *w0, double *w1)
{
    *k = 0; *w0 = 0.0; *w1 = 0.0;
    if (!(M > 0.0)) return;
    if (M >= m[N - 1]) { *k = N - 1; *w0 = M; return; }
    if (M < m[0]) { *k = 0; *w0 = M; return; }
    int l = 0;
    for (int q = 0; q < N; ++q)
        if (m[q] <= M) l = q;
    int u = l + 1;
    /* eps and 1 - eps, the latter written as (M - m_l)/(m_u - m_l) so that it
       does not cancel when M is close to m_l on a coarse grid */
    double eps = (m[u] - M) / (m[u] - m[l]);
    double ome = (M - m[l]) / (m[u] - m[l]);
    *k = l;
    if (split == ORACLE_SPLIT_NUMBER) {
        *w0 = eps * m[l];
        *w1 = ome * m[u];
    } else {
        *w0 = eps * M;
        *w1 = ome * M;
    }
}

int ored_build(const oracle_grid_t *g, ored *r)
{
    const int N = g->N;
    const long P = (long)N * (N + 1) / 2;
    memset(r, 0, sizeof(*r));
    r->N = N; r->P = P; r->m = g->m; r->m_edge = g->m_edge; r->s = g->s;
    r->rho_m = g->rho_m;
    r->vertical = g->vertical;
    r->ci = malloc(P * sizeof(int)); r->cw0 = malloc(P * sizeof(double)); r->cw1 = malloc(P * sizeof(double));
    r->ri = malloc(P * sizeof(int)); r->rw0 = malloc(P * sizeof(double)); r->rw1 = malloc(P * sizeof(double));
    r->fl = malloc(P * sizeof(int)); r->fm = malloc(P * sizeof(double));
    r->pi = malloc(P * sizeof(int)); r->pj = malloc(P * sizeof(int));
    r->Nfrac = calloc((size_t)N * N, sizeof(double));
    if (!r->ci || !r->cw0 || !r->cw1 || !r->ri || !r->rw0 || !r->rw1 || !r->fl ||
        !r->fm || !r->pi || !r->pj || !r->Nfrac) { ored_free(r); return -2; }

    const double *m = g->m, *me = g->m_edge;
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j <= i; ++j) {
            long p = (long)i * (i + 1) / 2 + j;
            r->pi[p] = i; r->pj[p] = j;
            /* coagulation: product mass m_i + m_j */
            split_mass(m, N, m[i] + m[j], g->split, &r->ci[p], &r->cw0[p], &r->cw1[p]);
            /* cratering (eq. `fragrem`): target i (the heavier), impactor j.
               The largest fragment is min(chi m_j, m_i); the fragment mass that
               is distributed is the total mass minus the remnant. */
            double m_rem, m_fmax;
            if (g->chi * m[j] < m[i]) {
                m_rem = m[i] - g->chi * m[j];
                m_fmax = g->chi * m[j];
            } else {
                m_rem = 0.0;
                m_fmax = m[i];
            }
            split_mass(m, N, m_rem, g->split, &r->ri[p], &r->rw0[p], &r->rw1[p]);
            r->fm[p] = (m[i] + m[j]) - m_rem;
            /* top fragment bin: smallest l with m^e_{l+1} > largest fragment */
            int l = N - 1;
            for (int q = N - 1; q >= 0; --q)
                if (me[q + 1] > m_fmax) l = q;
            r->fl[p] = l;
        }
    }
    /* power-law fragment mass fractions, eq. `Nijk`, for every top bin l */
    for (int l = 0; l < N; ++l) {
        double den = pow(me[l + 1], 2.0 - g->eta) - pow(me[0], 2.0 - g->eta);
        for (int k = 0; k <= l; ++k)
            r->Nfrac[(long)l * N + k] =
                (pow(me[k + 1], 2.0 - g->eta) - pow(me[k], 2.0 - g->eta)) / den;
    }
    return 0;
}

void ored_free(ored *r)
{
    free(r->ci); free(r->cw0); free(r->cw1);
    free(r->ri); free(r->rw0); free(r->rw1);
    free(r->fl); free(r->fm); free(r->pi); free(r->pj); free(r->Nfrac);
    memset(r, 0, sizeof(*r));
}

static int grid_ok(const oracle_grid_t *g)
{
    if (!g || g->N < 2 || !g->m || !g->m_edge || !g->s) return 0;
    if (!(g->chi > 0) || g->eta == 2.0 || !(g->rho_m > 0)) return 0;
    for (int k = 0; k + 1 < g->N; ++k) if (!(g->m[k + 1] > g->m[k])) return 0;
    for (int k = 0; k < g->N; ++k)
        if (!(g->m_edge[k] < g->m[k] && g->m[k] < g->m_edge[k + 1])) return 0;
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Exported: redistribution tables                                           */
/* ------------------------------------------------------------------------- */

/* Dense redistribution matrix D[2P][N] of the gain term (eq. `ngain`):
   row p      : (m_i + m_j) C_ijk                  (coagulating collisions)
   row P + p  : m_rem R_ijk + m_frag F_ijk         (fragmenting collisions)
   with F_ijk = N_k(m^e_{l+1}) written out per pair (no accumulation trick). */
int oracle_redistribution_dense(const oracle_grid_t *g, double *D)
{
    if (!grid_ok(g)) return -1;
    ored r;
    if (ored_build(g, &r)) return -2;
    const int N = r.N;
    const long P = r.P;
    memset(D, 0, sizeof(double) * 2 * P * N);
    for (long p = 0; p < P; ++p) {
        double *dc = D + p * N, *df = D + (P + p) * N;
        dc[r.ci[p]] += r.cw0[p];
        if (r.cw1[p] != 0.0) dc[r.ci[p] + 1] += r.cw1[p];
        if (r.rw0[p] != 0.0) df[r.ri[p]] += r.rw0[p];
        if (r.rw1[p] != 0.0) df[r.ri[p] + 1] += r.rw1[p];
        for (int k = 0; k <= r.fl[p]; ++k)
            df[k] += r.fm[p] * r.Nfrac[(long)r.fl[p] * N + k];
    }
    ored_free(&r);
    return 0;
}

/* Sparse per-pair tables, for inspection by tests. */
int oracle_redistribution_sparse(const oracle_grid_t *g, int32_t *ci, double *cw,
                                 int32_t *ri, double *rw, int32_t *fl, double *fm,
                                 double *Nfrac)
{
    if (!grid_ok(g)) return -1;
    ored r;
    if (ored_build(g, &r)) return -2;
    for (long p = 0; p < r.P; ++p) {
        ci[p] = r.ci[p]; cw[2 * p] = r.cw0[p]; cw[2 * p + 1] = r.cw1[p];
        ri[p] = r.ri[p]; rw[2 * p] = r.rw0[p]; rw[2 * p + 1] = r.rw1[p];
        fl[p] = r.fl[p]; fm[p] = r.fm[p];
    }
    memcpy(Nfrac, r.Nfrac, sizeof(double) * r.N * r.N);
    ored_free(&r);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Exported: rates and right-hand side                                       */
/* ------------------------------------------------------------------------- */
int oracle_rates(const oracle_grid_t *g, long C, const oracle_cells_t *c,
                 const double *v /* [C][N][3] */, const double *v_frag /* [C] */,
                 double *Kc, double *Kf)
{
    if (!grid_ok(g) || C < 0) return -1;
    ored r;
    memset(&r, 0, sizeof(r));
    r.N = g->N; r.P = (long)g->N * (g->N + 1) / 2;
    r.m = g->m; r.m_edge = g->m_edge; r.s = g->s; r.rho_m = g->rho_m;
    r.vertical = g->vertical;
    const int N = r.N;
    const long P = r.P;
#pragma omp parallel for schedule(dynamic, 4)
    for (long q = 0; q < C; ++q)
        r_rates_cell(&r, c->T[q], c->rho_g[q], c->c_s[q], c->Omega[q], c->H[q],
                     c->nu_mol[q], c->alpha[q], v + q * N * 3, v_frag[q],
                     Kc + q * P, Kf + q * P);
    return 0;
}

int oracle_rhs(const oracle_grid_t *g, long C, const double *rho, const double *Kc,
               const double *Kf, double *drho, double *gain, double *loss)
{
    if (!grid_ok(g) || C < 0) return -1;
    ored r;
    if (ored_build(g, &r)) return -2;
    const int N = r.N;
    const long P = r.P;
    int bad = 0;
#pragma omp parallel
    {
        double *w = malloc(sizeof(double) * 4 * N);
        if (!w) bad = 1;
#pragma omp for schedule(dynamic, 4)
        for (long q = 0; q < C; ++q)
            if (w) r_rhs_cell(&r, rho + q * N, Kc + q * P, Kf + q * P, drho + q * N,
                              gain ? gain + q * N : 0, loss ? loss + q * N : 0, w);
        free(w);
    }
    ored_free(&r);
    return bad ? -2 : 0;
}

/* RHS through the dense matrix D (literal per-pair F_ijk): the same quantity
   as oracle_rhs, evaluated as gain = [Rc | Rf] . D. */
int oracle_rhs_dense(const oracle_grid_t *g, long C, const double *rho, const double *Kc,
                     const double *Kf, double *drho)
{
    if (!grid_ok(g) || C < 0) return -1;
    const int N = g->N;
    const long P = (long)N * (N + 1) / 2;
    double *D = malloc(sizeof(double) * 2 * P * N);
    if (!D) return -2;
    int rc = oracle_redistribution_dense(g, D);
    if (rc) { free(D); return rc; }
    for (long q = 0; q < C; ++q) {
        const double *y = rho + q * N, *kc = Kc + q * P, *kf = Kf + q * P;
        double *out = drho + q * N;
        double *n = malloc(sizeof(double) * N);
        for (int k = 0; k < N; ++k) { n[k] = y[k] / g->m[k]; out[k] = 0.0; }
        for (int i = 0; i < N; ++i)
            for (int j = 0; j <= i; ++j) {
                long p = (long)i * (i + 1) / 2 + j;
                double Rc = n[i] * n[j] * kc[p], Rf = n[i] * n[j] * kf[p];
                for (int k = 0; k < N; ++k)
                    out[k] += Rc * D[p * N + k] + Rf * D[(P + p) * N + k];
                /* loss of both partners (once on the diagonal, un-halved kernel) */
                double w = (i == j) ? 0.5 : 1.0;
                double Kt = (kc[p] + kf[p]) / w;
                out[i] -= g->m[i] * n[i] * Kt * n[j];
                if (i != j) out[j] -= g->m[j] * n[j] * Kt * n[i];
            }
        free(n);
    }
    free(D);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Exported: the time step (Sec. 5 closing paragraph; Sec. 6 sub-cycling).   */
/*                                                                           */
/* Per cell, integrate drho/dt = f(rho) over dt with BS3(2):                  */
/*   ADAPTIVE: error e = h(-5/72 k1 + 1/12 k2 + 1/9 k3 - 1/8 k4), scaled by   */
/*     sc_k = atol + rtol max(|y_k|, |y+_k|), atol = atol_rel * sum_k y_k at  */
/*     entry; err = max_k |e_k| / sc_k.  Accept iff err <= 1 and no state     */
/*     below -atol.  Step factor clamp(0.9 err^(-1/3), 0.2, 5) (5 if err=0),  */
/*     0.5 for a rejection caused only by a negative state.  The last step    */
/*     is clipped to land on dt; a clipped accepted step leaves the proposed  */
/*     h unchanged, so h on exit is the controller's next unclipped step.     */
/*   FIXED   : nsub[c] equal steps of dt / nsub[c], all accepted.            */
/*   REPLAY  : nsub[c] accepted steps of the sizes in h_log[c][:].           */
/* h[c] <= 0 on entry means "start with dt".  nacc/nrej count accepted and    */
/* rejected attempts; h_log (may be NULL in FIXED mode) records accepted step */
/* sizes, max_sub entries per cell.                                          */
/* ------------------------------------------------------------------------- */
static int step_cell(const ored *r, double *y, const double *Kc, const double *Kf,
                     double dt, double *h_io, const oracle_tol_t *tol,
                     int *nacc_io, int *nrej, double *hlog, double *w)
{
    const int N = r->N;
    double *k1 = w, *k2 = w + N, *k3 = w + 2 * N, *k4 = w + 3 * N;
    double *ys = w + 4 * N, *yn = w + 5 * N, *wk = w + 6 * N;
    int nacc = 0;
    *nrej = 0;
    r_rhs_cell(r, y, Kc, Kf, k1, 0, 0, wk);

    if (tol->mode == ORACLE_FIXED || tol->mode == ORACLE_REPLAY) {
        int n = *nacc_io;
        for (int s = 0; s < n; ++s) {
            double hh = tol->mode == ORACLE_FIXED ? dt / n : hlog[s];
            r_bs3_advance(r, y, k1, hh, Kc, Kf, ys);
            r_rhs_cell(r, y, Kc, Kf, k1, 0, 0, wk);
            if (tol->mode == ORACLE_FIXED && hlog) hlog[s] = hh;
        }
        for (int k = 0; k < N; ++k) if (!isfinite(y[k])) return ORACLE_CELL_NONFINITE;
        return ORACLE_CELL_OK;
    }

    double mass = 0.0;
    for (int k = 0; k < N; ++k) mass += y[k];
    const double atol = tol->atol_rel * mass;
    double h = *h_io > 0.0 ? *h_io : dt;
    double t = 0.0;
    int status = ORACLE_CELL_OK;
    while (t < dt) {
        if (nacc + *nrej >= tol->max_sub) { status = ORACLE_CELL_MAXSUB; break; }
        double hh = h;
        int clipped = 0;
        if (hh >= dt - t) { hh = dt - t; clipped = 1; }
        if (!clipped && hh < tol->h_min_rel * dt) { status = ORACLE_CELL_HMIN; break; }
        for (int k = 0; k < N; ++k) ys[k] = y[k] + 0.5 * hh * k1[k];
        r_rhs_cell(r, ys, Kc, Kf, k2, 0, 0, wk);
        for (int k = 0; k < N; ++k) ys[k] = y[k] + 0.75 * hh * k2[k];
        r_rhs_cell(r, ys, Kc, Kf, k3, 0, 0, wk);
        for (int k = 0; k < N; ++k)
            yn[k] = y[k] + hh * (2.0 / 9.0 * k1[k] + 1.0 / 3.0 * k2[k] + 4.0 / 9.0 * k3[k]);
        r_rhs_cell(r, yn, Kc, Kf, k4, 0, 0, wk);
        double err = 0.0;
        int neg = 0, finite = 1;
        for (int k = 0; k < N; ++k) {
            double e = hh * (-5.0 / 72.0 * k1[k] + 1.0 / 12.0 * k2[k]
                             + 1.0 / 9.0 * k3[k] - 1.0 / 8.0 * k4[k]);
            double ay = fabs(y[k]), ayn = fabs(yn[k]);
            double sc = atol + tol->rtol * (ay > ayn ? ay : ayn);
            double q = fabs(e) / sc;
            if (q > err) err = q;
            if (yn[k] < -atol) neg = 1;
            if (!isfinite(yn[k]) || !isfinite(e)) finite = 0;
        }
        if (!finite || !isfinite(err)) { status = ORACLE_CELL_NONFINITE; break; }
        double fac = err == 0.0 ? 5.0 : 0.9 * pow(err, -1.0 / 3.0);
        if (fac < 0.2) fac = 0.2;
        if (fac > 5.0) fac = 5.0;
        if (err <= 1.0 && !neg) {
            if (hlog && nacc < tol->max_sub) hlog[nacc] = hh;
            ++nacc;
            t = clipped ? dt : t + hh;
            memcpy(y, yn, sizeof(double) * N);
            memcpy(k1, k4, sizeof(double) * N);
            if (!clipped) h = hh * fac;
        } else {
            ++*nrej;
            h = hh * (err <= 1.0 ? 0.5 : fac);
        }
    }
    *h_io = h;
    *nacc_io = nacc;
    return status;
}

int oracle_step(const oracle_grid_t *g, long C, double *rho, const double *Kc,
                const double *Kf, double dt, double *h, const oracle_tol_t *tol,
                int32_t *nsub, int32_t *nrej, double *h_log, int32_t *status)
{
    if (!grid_ok(g) || C < 0 || !(dt > 0) || !tol || !(tol->rtol > 0) || tol->max_sub < 1)
        return -1;
    if (tol->mode == ORACLE_REPLAY && !h_log) return -1;
    ored r;
    if (ored_build(g, &r)) return -2;
    const int N = r.N;
    const long P = r.P;
    int bad = 0;
#pragma omp parallel
    {
        double *w = malloc(sizeof(double) * 12 * N);
        if (!w) bad = 1;
#pragma omp for schedule(dynamic, 1)
        for (long q = 0; q < C; ++q) {
            if (!w) continue;
            int na = (tol->mode == ORACLE_ADAPTIVE) ? 0 : nsub[q];
            int nr = 0;
            double hq = h ? h[q] : 0.0;
            int st = step_cell(&r, rho + q * N, Kc + q * P, Kf + q * P, dt, &hq, tol,
                               &na, &nr, h_log ? h_log + q * (long)tol->max_sub : 0, w);
            if (h && tol->mode == ORACLE_ADAPTIVE) h[q] = hq;
            nsub[q] = na;
            if (nrej) nrej[q] = nr;
            if (status) status[q] = st;
        }
        free(w);
    }
    ored_free(&r);
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------------- */
/* Hand-written discrete adjoint.                                            */
/* ------------------------------------------------------------------------- */

/* Derivatives of Kc, Kf with respect to alpha and v_frag for one cell,
   differentiating the rate formulas of rates_cell by hand.  The clamps of St*
   and the p_coag branch are taken as in the forward pass. */
static void rates_cell_deriv(const ored *r, double Tgas, double rho_g, double c_s,
                             double Omega, double H, double nu_mol, double alpha,
                             const double *v, double v_frag,
                             double *dKc_da, double *dKf_da, double *dKc_dv, double *dKf_dv)
{
    const int N = r->N;
    const double *m = r->m, *s = r->s;
    const double v_th = sqrt(8.0 / M_PI) * c_s;
    double Re = alpha * c_s * H / nu_mol;
    double delta = 1.0 / sqrt(Re);
    double ddelta_da = -0.5 * delta / alpha;      /* delta ~ alpha^(-1/2) */
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j <= i; ++j) {
            long p = (long)i * (i + 1) / 2 + j;
            double St_i = r->rho_m * s[i] / (rho_g * v_th) * Omega;
            double St_j = r->rho_m * s[j] / (rho_g * v_th) * Omega;
            double St1 = St_i >= St_j ? St_i : St_j;
            double St2 = St_i >= St_j ? St_j : St_i;
            double S = ORACLE_YSTAR * St1;
            double dS_ddelta = 0.0;
            if (S < delta) { S = delta; dS_ddelta = 1.0; }
            if (S > 1.0) { S = 1.0; dS_ddelta = 0.0; }
            double f12 = (St1 - St2) / (St1 + St2);
            double dV1 = f12 * (St1 * St1 / (S + St1) - St1 * St1 / (1.0 + St1)
                                - St2 * St2 / (S + St2) + St2 * St2 / (1.0 + St2));
            double dV2 = 2.0 * (S - delta)
                         + St1 * St1 / (St1 + S) - St1 * St1 / (St1 + delta)
                         + St2 * St2 / (St2 + S) - St2 * St2 / (St2 + delta);
            double Vrel2 = dV1 + dV2;
            /* d/dS and d/ddelta of the class I + II sum */
            double dV_dS = f12 * (-St1 * St1 / ((S + St1) * (S + St1))
                                  + St2 * St2 / ((S + St2) * (S + St2)))
                           + 2.0 - St1 * St1 / ((St1 + S) * (St1 + S))
                           - St2 * St2 / ((St2 + S) * (St2 + S));
            double dV_ddelta = -2.0 + St1 * St1 / ((St1 + delta) * (St1 + delta))
                               + St2 * St2 / ((St2 + delta) * (St2 + delta));
            double dVrel2_da = (dV_ddelta + dV_dS * dS_ddelta) * ddelta_da;

            double vturb2 = alpha > 0.0 ? alpha * c_s * c_s * Vrel2 : 0.0;
            double dvturb2_da = alpha > 0.0 ? c_s * c_s * Vrel2 + alpha * c_s * c_s * dVrel2_da : 0.0;
            double vbm2 = 8.0 * ORACLE_KB * Tgas * (m[i] + m[j]) / (M_PI * m[i] * m[j]);
            double dx = v[3 * i + 0] - v[3 * j + 0];
            double dy = v[3 * i + 1] - v[3 * j + 1];
            double dz = v[3 * i + 2] - v[3 * j + 2];
            /* vertically integrated kernel: h_k = H sqrt(alpha / (alpha + St_k))
               has d ln h_k / d alpha = St_k / (2 alpha (alpha + St_k)) = e_k; the
               settling speeds St_k Omega h_k and the overlap factor
               G = (2 pi (h_i^2 + h_j^2))^(-1/2) move with alpha through h */
            double G = 1.0, dlnG_da = 0.0, dvlam2_da = 0.0;
            if (r->vertical) {
                double h_i = H * sqrt(alpha / (alpha + St_i));
                double h_j = H * sqrt(alpha / (alpha + St_j));
                double e_i = St_i / (2.0 * alpha * (alpha + St_i));
                double e_j = St_j / (2.0 * alpha * (alpha + St_j));
                double vz_i = St_i * Omega * h_i, vz_j = St_j * Omega * h_j;
                dz = vz_i - vz_j;
                dvlam2_da = 2.0 * dz * (vz_i * e_i - vz_j * e_j);
                double hh = h_i * h_i + h_j * h_j;
                G = 1.0 / sqrt(2.0 * M_PI * hh);
                dlnG_da = -(h_i * h_i * e_i + h_j * h_j * e_j) / hh;
            }
            double vlam2 = dx * dx + dy * dy + dz * dz;
            double dv = sqrt(vbm2 + vturb2 + vlam2);
            double ddv_da = (dvturb2_da + dvlam2_da) / (2.0 * dv);
            double sig = M_PI * (s[i] + s[j]) * (s[i] + s[j]);
            double K = sig * dv * G;
            double w = (i == j) ? 0.5 : 1.0;

            double pf, pc, dpf_dy;
            double y = 0.0;
            if (dv == 0.0) {
                pf = 0.0; pc = 1.0; dpf_dy = 0.0;
            } else {
                y = 1.5 * (v_frag / dv) * (v_frag / dv);
                double e = exp(-y);
                pf = (1.0 + y) * e;
                if (y < ORACLE_PSERIES_Y) {
                    double y2 = y * y;
                    pc = y2 * (1.0 / 2.0 + y * (-1.0 / 3.0 + y * (1.0 / 8.0 + y * (-1.0 / 30.0
                         + y * (1.0 / 144.0 + y * (-1.0 / 840.0 + y * (1.0 / 5760.0)))))));
                } else {
                    pc = 1.0 - pf;
                }
                dpf_dy = -y * e;                     /* d/dy [(1+y) e^-y] */
            }
            /* dy/dv_frag = 3 v_frag / dv^2 ; dy/ddv = -2 y / dv */
            double dy_dvf = dv > 0 ? 3.0 * v_frag / (dv * dv) : 0.0;
            double dy_ddv = dv > 0 ? -2.0 * y / dv : 0.0;
            double dpf_ddv = dpf_dy * dy_ddv;
            /* Kc = w sig dv G pc, Kf = w sig dv G pf, pc = 1 - pf */
            dKf_da[p] = w * (sig * G * pf + K * dpf_ddv) * ddv_da + w * K * pf * dlnG_da;
            dKc_da[p] = w * (sig * G * pc - K * dpf_ddv) * ddv_da + w * K * pc * dlnG_da;
            dKf_dv[p] = w * K * dpf_dy * dy_dvf;
            dKc_dv[p] = -dKf_dv[p];
        }
    }
}

/* Vector-Jacobian product of the right-hand side for one cell:
   given mu = dJ/d(drho), accumulate dJ/drho into gy and dJ/dKc, dJ/dKf into
   gKc, gKf.  The gain is bilinear in n and the rates, so with a_p = n_i n_j
     drho = sum_p a_p (Kc_p (Dc_p - l_p) + Kf_p (Df_p - l_p))
   where Dc_p, Df_p are the redistribution rows of eq. `ngain` and l_p holds
   the two partners' loss masses m_i, m_j divided by w_p (once on the
   diagonal). */
static void vjp_rhs_cell(const ored *r, const double *rho, const double *Kc,
                         const double *Kf, const double *mu, double *gy,
                         double *gKc, double *gKf, double *w /* 3N */)
{
    const int N = r->N;
    const double *m = r->m;
    double *n = w, *gn = w + N, *suf = w + 2 * N;
    for (int k = 0; k < N; ++k) { n[k] = rho[k] / m[k]; gn[k] = 0.0; }
    /* fragment part of mu . Df_p : m_frag sum_{k<=l} mu_k N_k(m^e_{l+1}) */
    for (int l = 0; l < N; ++l) {
        double acc = 0.0;
        for (int k = 0; k <= l; ++k) acc += mu[k] * r->Nfrac[(long)l * N + k];
        suf[l] = acc;
    }
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j <= i; ++j) {
            long p = (long)i * (i + 1) / 2 + j;
            double wp = (i == j) ? 0.5 : 1.0;
            double lp = (i == j) ? mu[i] * m[i] / wp : (mu[i] * m[i] + mu[j] * m[j]) / wp;
            double dc = mu[r->ci[p]] * r->cw0[p]
                        + (r->cw1[p] != 0.0 ? mu[r->ci[p] + 1] * r->cw1[p] : 0.0);
            double df = (r->rw0[p] != 0.0 ? mu[r->ri[p]] * r->rw0[p] : 0.0)
                        + (r->rw1[p] != 0.0 ? mu[r->ri[p] + 1] * r->rw1[p] : 0.0)
                        + r->fm[p] * suf[r->fl[p]];
            double sc = dc - lp, sf = df - lp;
            double a = n[i] * n[j];
            double ga = Kc[p] * sc + Kf[p] * sf;
            gKc[p] += a * sc;
            gKf[p] += a * sf;
            gn[i] += n[j] * ga;
            gn[j] += n[i] * ga;
        }
    }
    for (int k = 0; k < N; ++k) gy[k] += gn[k] / m[k];
}

/* Adjoint of `nsub[c]` accepted BS3 steps with sizes h_log[c][:] (a frozen
   step sequence, as REPLAY or FIXED reproduce it), including the rates'
   dependence on alpha and v_frag.  g_out = dJ/drho(final); outputs
   g_in = dJ/drho(start), g_alpha[c] = dJ/dalpha_c, g_vfrag[c] = dJ/dv_frag,c.
   Reverse sweep of the stage recurrences:
     mu3 = h b3 lam,              v3 = J(y3)^T mu3
     mu2 = h b2 lam + 3h/4 v3,    v2 = J(y2)^T mu2
     mu1 = h b1 lam + h/2 v2,     v1 = J(y)^T mu1
     lam <- lam + v1 + v2 + v3.                                             */
int oracle_step_backward(const oracle_grid_t *g, long C, const oracle_cells_t *c,
                         const double *v, const double *v_frag, const double *rho_in,
                         double dt, const double *h_log, const int32_t *nsub,
                         int32_t log_stride, const double *g_out, double *g_in,
                         double *g_alpha, double *g_vfrag)
{
    (void)dt;
    if (!grid_ok(g) || C < 0 || !h_log || !nsub || log_stride < 1) return -1;
    ored r;
    if (ored_build(g, &r)) return -2;
    const int N = r.N;
    const long P = r.P;
    int bad = 0;
#pragma omp parallel
    {
        double *Kc = malloc(sizeof(double) * 6 * P);
        double *w = malloc(sizeof(double) * 16 * N);
        if (!Kc || !w) bad = 1;
#pragma omp for schedule(dynamic, 1)
        for (long q = 0; q < C; ++q) {
            if (!Kc || !w) continue;
            double *Kf = Kc + P, *gKc = Kc + 2 * P, *gKf = Kc + 3 * P;
            double *dKc_da = Kc + 4 * P, *dKf_da = Kc + 5 * P;
            const int ns = nsub[q];
            const double *hl = h_log + q * (long)log_stride;
            r_rates_cell(&r, c->T[q], c->rho_g[q], c->c_s[q], c->Omega[q], c->H[q],
                         c->nu_mol[q], c->alpha[q], v + q * N * 3, v_frag[q], Kc, Kf);
            double *ys = malloc(sizeof(double) * (size_t)(ns + 1) * N);
            if (!ys) { bad = 1; continue; }
            double *k1 = w, *y2 = w + N, *y3 = w + 2 * N, *kk = w + 3 * N;
            double *lam = w + 4 * N, *mu = w + 5 * N, *vv = w + 6 * N, *vtmp = w + 7 * N;
            double *wk = w + 8 * N;
            /* forward: states at the start of each accepted step */
            memcpy(ys, rho_in + q * N, sizeof(double) * N);
            for (int s = 0; s < ns; ++s) {
                memcpy(ys + (size_t)(s + 1) * N, ys + (size_t)s * N, sizeof(double) * N);
                r_rhs_cell(&r, ys + (size_t)s * N, Kc, Kf, k1, 0, 0, wk);
                r_bs3_advance(&r, ys + (size_t)(s + 1) * N, k1, hl[s], Kc, Kf, wk);
            }
            memset(gKc, 0, sizeof(double) * 2 * P);
            memcpy(lam, g_out + q * N, sizeof(double) * N);
            for (int s = ns - 1; s >= 0; --s) {
                const double h = hl[s];
                const double *y = ys + (size_t)s * N;
                r_rhs_cell(&r, y, Kc, Kf, k1, 0, 0, wk);
                for (int k = 0; k < N; ++k) y2[k] = y[k] + 0.5 * h * k1[k];
                r_rhs_cell(&r, y2, Kc, Kf, kk, 0, 0, wk);
                for (int k = 0; k < N; ++k) y3[k] = y[k] + 0.75 * h * kk[k];
                /* stage 3 */
                for (int k = 0; k < N; ++k) { mu[k] = h * 4.0 / 9.0 * lam[k]; vv[k] = 0.0; }
                vjp_rhs_cell(&r, y3, Kc, Kf, mu, vv, gKc, gKf, wk);
                /* stage 2 */
                for (int k = 0; k < N; ++k) { mu[k] = h / 3.0 * lam[k] + 0.75 * h * vv[k]; vtmp[k] = 0.0; }
                vjp_rhs_cell(&r, y2, Kc, Kf, mu, vtmp, gKc, gKf, wk);
                /* stage 1 */
                for (int k = 0; k < N; ++k) {
                    mu[k] = h * 2.0 / 9.0 * lam[k] + 0.5 * h * vtmp[k];
                    lam[k] += vv[k] + vtmp[k];
                }
                for (int k = 0; k < N; ++k) vv[k] = 0.0;
                vjp_rhs_cell(&r, y, Kc, Kf, mu, vv, gKc, gKf, wk);
                for (int k = 0; k < N; ++k) lam[k] += vv[k];
            }
            memcpy(g_in + q * N, lam, sizeof(double) * N);
            /* chain through the rates: reuse Kc/Kf storage for dK/dv_frag */
            double *dKc_dv = Kc, *dKf_dv = Kf;
            rates_cell_deriv(&r, c->T[q], c->rho_g[q], c->c_s[q], c->Omega[q], c->H[q],
                             c->nu_mol[q], c->alpha[q], v + q * N * 3, v_frag[q],
                             dKc_da, dKf_da, dKc_dv, dKf_dv);
            double ga = 0.0, gv = 0.0;
            for (long p = 0; p < P; ++p) {
                ga += gKc[p] * dKc_da[p] + gKf[p] * dKf_da[p];
                gv += gKc[p] * dKc_dv[p] + gKf[p] * dKf_dv[p];
            }
            g_alpha[q] = ga;
            g_vfrag[q] = gv;
            free(ys);
        }
        free(Kc);
        free(w);
    }
    ored_free(&r);
    return bad ? -2 : 0;
}

/* VJP of the right-hand side alone (for tests): gy = J^T mu, gKc, gKf. */
int oracle_rhs_vjp(const oracle_grid_t *g, long C, const double *rho, const double *Kc,
                   const double *Kf, const double *mu, double *gy, double *gKc, double *gKf)
{
    if (!grid_ok(g) || C < 0) return -1;
    ored r;
    if (ored_build(g, &r)) return -2;
    const int N = r.N;
    const long P = r.P;
    double *w = malloc(sizeof(double) * 3 * N);
    if (!w) { ored_free(&r); return -2; }
    for (long q = 0; q < C; ++q) {
        memset(gy + q * N, 0, sizeof(double) * N);
        memset(gKc + q * P, 0, sizeof(double) * P);
        memset(gKf + q * P, 0, sizeof(double) * P);
        vjp_rhs_cell(&r, rho + q * N, Kc + q * P, Kf + q * P, mu + q * N, gy + q * N,
                     gKc + q * P, gKf + q * P, w);
    }
    free(w);
    ored_free(&r);
    return 0;
}

/* Rate derivatives (for tests). */
int oracle_rates_deriv(const oracle_grid_t *g, long C, const oracle_cells_t *c,
                       const double *v, const double *v_frag, double *dKc_da,
                       double *dKf_da, double *dKc_dv, double *dKf_dv)
{
    if (!grid_ok(g) || C < 0) return -1;
    ored r;
    memset(&r, 0, sizeof(r));
    r.N = g->N; r.P = (long)g->N * (g->N + 1) / 2;
    r.m = g->m; r.m_edge = g->m_edge; r.s = g->s; r.rho_m = g->rho_m;
    r.vertical = g->vertical;
    const long P = r.P;
    for (long q = 0; q < C; ++q)
        rates_cell_deriv(&r, c->T[q], c->rho_g[q], c->c_s[q], c->Omega[q], c->H[q],
                         c->nu_mol[q], c->alpha[q], v + q * r.N * 3, v_frag[q],
                         dKc_da + q * P, dKf_da + q * P, dKc_dv + q * P, dKf_dv + q * P);
    return 0;
}

/* Threads the OpenMP loops over cells use from now on (n >= 1); for the
   single-thread timing of the CPU baseline. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
