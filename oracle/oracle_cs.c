/*
 * oracle_cs.c -- complex-step derivatives of the oracle's forward arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).  The same forward formulas as the
 * FP64 oracle are instantiated over double complex; a perturbation i*hcs of
 * one input gives dJ/dx = Im(J)/hcs to machine precision (no subtractive
 * cancellation), independently of the hand-written adjoint in oracle.c.
 * Branches and clamps are decided on real parts, so the derivative is the
 * one-sided derivative of the branch the forward pass takes.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle_core.h"

#define SC double complex
#define FN(name) c_##name
#define RE(x) creal(x)
#define SQRTT(x) csqrt(x)
#define EXPT(x) cexp(x)
#include "oracle_fwd.inc"

/* J = sum_c sum_k g_out[c][k] rho_final[c][k] after the frozen step sequence
   (nsub[c] steps of sizes h_log[c][:]) from rho_in, with rates computed from
   the cell state.  One input is perturbed by i*hcs:
     which = 0 : rho_in[index]  (flat index over [C][N])
     which = 1 : alpha[index]   (cell index)
     which = 2 : v_frag[index]  (cell index)
   Returns dJ/d(input). */
double oracle_cs_step_grad(const oracle_grid_t *g, long C, const oracle_cells_t *c,
                           const double *v, const double *v_frag, const double *rho_in,
                           const double *h_log, const int32_t *nsub, int32_t log_stride,
                           const double *g_out, int which, long index, double hcs)
{
    ored r;
    if (ored_build(g, &r)) return NAN;
    const int N = r.N;
    const long P = r.P;
    SC *Kc = malloc(sizeof(SC) * 2 * P), *Kf;
    SC *y = malloc(sizeof(SC) * 14 * N);
    if (!Kc || !y) { free(Kc); free(y); ored_free(&r); return NAN; }
    Kf = Kc + P;
    SC *k1 = y + N, *wk = y + 2 * N;
    SC J = 0.0;
    for (long q = 0; q < C; ++q) {
        SC alpha = c->alpha[q], vf = v_frag[q];
        if (which == 1 && index == q) alpha += I * hcs;
        if (which == 2 && index == q) vf += I * hcs;
        c_rates_cell(&r, c->T[q], c->rho_g[q], c->c_s[q], c->Omega[q], c->H[q],
                     c->nu_mol[q], alpha, v + q * N * 3, vf, Kc, Kf);
        for (int k = 0; k < N; ++k) {
            y[k] = rho_in[q * N + k];
            if (which == 0 && index == q * N + k) y[k] += I * hcs;
        }
        const double *hl = h_log + q * (long)log_stride;
        for (int s = 0; s < nsub[q]; ++s) {
            c_rhs_cell(&r, y, Kc, Kf, k1, 0, 0, wk);
            c_bs3_advance(&r, y, k1, hl[s], Kc, Kf, wk);
        }
        for (int k = 0; k < N; ++k) J += g_out[q * N + k] * y[k];
    }
    free(Kc);
    free(y);
    ored_free(&r);
    return cimag(J) / hcs;
}

/* J = mu . f(rho) for one cell with one perturbed input:
     which = 0 : rho[index], 3 : Kc[index], 4 : Kf[index].  Returns dJ/d(input). */
double oracle_cs_rhs_grad(const oracle_grid_t *g, const double *rho, const double *Kc_in,
                          const double *Kf_in, const double *mu, int which, long index,
                          double hcs)
{
    ored r;
    if (ored_build(g, &r)) return NAN;
    const int N = r.N;
    const long P = r.P;
    SC *Kc = malloc(sizeof(SC) * 2 * P), *Kf;
    SC *y = malloc(sizeof(SC) * 6 * N);
    if (!Kc || !y) { free(Kc); free(y); ored_free(&r); return NAN; }
    Kf = Kc + P;
    for (long p = 0; p < P; ++p) { Kc[p] = Kc_in[p]; Kf[p] = Kf_in[p]; }
    if (which == 3) Kc[index] += I * hcs;
    if (which == 4) Kf[index] += I * hcs;
    for (int k = 0; k < N; ++k) y[k] = rho[k];
    if (which == 0) y[index] += I * hcs;
    SC *f = y + N, *wk = y + 2 * N;
    c_rhs_cell(&r, y, Kc, Kf, f, 0, 0, wk);
    SC J = 0.0;
    for (int k = 0; k < N; ++k) J += mu[k] * f[k];
    free(Kc);
    free(y);
    ored_free(&r);
    return cimag(J) / hcs;
}
