// coag_transport.hip -- the dust transport step of the dynamics solver
// (Sec. 3) on the cylinder/cone grid of Sec. 7, and the scheduler of Sec. 6
// that calls the coagulation update from the transport's global steps.
//
// One thread per (cell, species): consecutive threads are the species of one
// cell, so every load of the state [C][N], [C][N][3] is contiguous over a
// wave and a cell's neighbours (c +- 1, c +- n_z) are whole contiguous rows.
// Each thread evaluates the fluxes through its own cell's four faces (a face
// shared by two cells is evaluated by both, from the same operands in the
// same order, hence to the same bits: the update stays conservative without
// a separate face pass or atomics).  The step is held by the issue and
// latency of its FP64 vector work: per (cell, species) the two kernels
// evaluate eight face fluxes (four per stage) with their square roots and,
// in the second stage, six limited slopes of four primitives each; whatever
// depends on the cell alone (geometry, gas, diffusion coefficients of the
// faces, reciprocals) comes from tables, read through the scalar cache.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/coag.h"
#include "../../include/coag_transport.h"
#include "coag_launch.h"
#include "coag_rate.h"

namespace coag {

// number of bins of a coagulation context, and whether its step takes
// 16-cell-blocked rates in a precision (coag_api.hip)
int ctx_bins(const ::coag_ctx *ctx);
bool ctx_blocked(const ::coag_ctx *ctx, int prec);
bool ctx_vertical(const ::coag_ctx *ctx);

namespace {

constexpr int kTBlock = 256;

// geometry of the grid (device arrays, see coag_transport.h)
struct TGeo {
    int nr, nz, N;
    const double *Rc;        // [nr] cell-centre radius sqrt(R- R+)
    const double *Re;        // [nr + 1] cylinder faces
    const double *dR;        // [nr] radial width
    const double *Rcone;     // [nr] area-weighted radius of ring i's cone faces
    const double *Rx;        // [nr + 4] radial coordinate of cells -2 .. nr + 1 (ghosts mirrored about the edges)
    const double *tc;        // [nz] cell-centre t
    const double *te;        // [nz + 1] cone faces
    const double *tx;        // [nz + 4] t of cells -2 .. nz + 1 (mirrored about the midplane and the top)
    const double *V;         // [nr * nz]
    const double *AR;        // [(nr + 1) * nz] cylinder-face areas
    const double *At;        // [nr * (nz + 1)] cone-face areas
    const double *s;         // [N] grain radii
    const double *iRc;       // [nr] 1 / R_c
    const double *irx;       // [nr + 3] 1 / (Rx[k+1] - Rx[k]), k = -2 .. nr
    const double *itx;       // [nz + 3] 1 / (tx[k+1] - tx[k]), k = -2 .. nz
    const double *nRt;       // [nz + 1] unit normal of cone face j: (nRt, nZt) = (-t, 1) / sqrt(1 + t^2)
    const double *nZt;       // [nz + 1]
    const double *iV;        // [nr * nz] 1 / V
    const double *om2;       // [nr * nz] GM / r^3 at the cell centre
    double rho_m, GM, Sc;
    double eps_floor;        // dust-to-gas floor (0: none)
};

// per-step tables of the gas (k_tr_prep): 1 / rho_g, the stopping time per
// unit grain radius, and each face's diffusion coefficient over the distance
// between the cells it joins (0 at the grid's outer faces and the midplane)
struct GasT {
    const double *irg;       // [C]
    const double *tsf;       // [C] t_stop / s
    const double *KR;        // [(nr + 1) * nz] cylinder faces
    const double *Kt;        // [nr * (nz + 1)] cone faces
    const double *v_g;       // [C][3]
    const double *rho_g;     // [C]
};

struct Gas {
    const double *rho_g, *c_s, *H, *alpha, *v_g;
};

struct Prim {
    double r, vR, vp, vZ;
};

// a cell's primitive state with the boundary rules: zero-gradient copies past
// the radial edges and the top, the mirror image (v_Z reversed) below the
// midplane
__device__ inline Prim fetch(const TGeo &g, const double *rho, const double *v, int i, int j,
                             int s) {
    const bool mir = j < 0;
    const int ii = i < 0 ? 0 : (i >= g.nr ? g.nr - 1 : i);
    const int jj = mir ? min(-j - 1, g.nz - 1) : min(j, g.nz - 1);
    const long k = ((long)ii * g.nz + jj) * g.N + s;
    Prim p;
    p.r = rho[k];
    p.vR = v[3 * k];
    p.vp = v[3 * k + 1];
    p.vZ = mir ? -v[3 * k + 2] : v[3 * k + 2];
    return p;
}

// van Leer's harmonic mean of two one-sided gradients (0 where they differ in
// sign).  Where a b > 0 in FP64, |a + b| >= sqrt(a b) is normal, so the refined
// hardware reciprocal of div_nr applies.
__device__ inline double vanleer(double a, double b) {
    return a * b > 0.0 ? div_nr(2.0 * a * b, a + b) : 0.0;
}

// limited slope of each primitive of cell m from its neighbours l and r;
// il, ir the inverse distances m - l and r - m
__device__ inline Prim slope(const Prim &l, const Prim &m, const Prim &r, double il, double ir) {
    Prim g;
    g.r = vanleer((m.r - l.r) * il, (r.r - m.r) * ir);
    g.vR = vanleer((m.vR - l.vR) * il, (r.vR - m.vR) * ir);
    g.vp = vanleer((m.vp - l.vp) * il, (r.vp - m.vp) * ir);
    g.vZ = vanleer((m.vZ - l.vZ) * il, (r.vZ - m.vZ) * ir);
    return g;
}

__device__ inline Prim extrap(const Prim &p, const Prim &g, double d) {
    return Prim{p.r + g.r * d, p.vR + g.vR * d, p.vp + g.vp * d, p.vZ + g.vZ * d};
}

// Flux (per unit area) of the four conserved quantities through a face of
// unit normal (nR, nZ) from the left and right states: the upwind flux of
// eq. `riemann` chosen by the Roe-averaged normal speed (eq. `roeav`; no
// flux where the two states move apart), plus the diffusive mass flux Fd
// carrying the advected quantities per unit mass (1, v_R, v_phi Rq, v_Z) of
// the state on its upwind side.  Rq: the face's radius of angular momentum.
__device__ inline void face_flux(const Prim &L, const Prim &R, double nR, double nZ, double Rq,
                                 double Fd, double F[4]) {
    // No fused multiply-adds here: at the midplane the two states are mirror
    // images (v_l = -v_r, equal densities), where the Roe speed is exactly 0
    // and the flux the reflecting mean, with no mass through the face; a
    // fused s_l v_l + s_r v_r leaves a rounding residue whose sign would pick
    // one side and let mass through.  The sign of the Roe speed is taken from
    // the two separately rounded products, which a comparison cannot fuse.
#pragma clang fp contract(off)
    const double vl = nR * L.vR + nZ * L.vZ, vr = nR * R.vR + nZ * R.vZ;
    const double ql[4] = {L.r, L.r * L.vR, L.r * L.vp * Rq, L.r * L.vZ};
    const double qr[4] = {R.r, R.r * R.vR, R.r * R.vp * Rq, R.r * R.vZ};
    const double sl = sqrt(fmax(L.r, 0.0)), sr = sqrt(fmax(R.r, 0.0));
    const double pl = sl * vl, pr = sr * vr;
    const int side = sl + sr > 0.0 ? (pl > -pr ? 1 : (pl < -pr ? -1 : 0)) : 0;
    const bool apart = vl < 0.0 && vr > 0.0;
    const double wl[4] = {1.0, L.vR, L.vp * Rq, L.vZ};
    const double wr[4] = {1.0, R.vR, R.vp * Rq, R.vZ};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double fl = ql[k] * vl, fr = qr[k] * vr;
        double f = side > 0 ? fl : (side < 0 ? fr : 0.5 * (fl + fr));
        if (apart) f = 0.0;
        F[k] = f + Fd * (Fd > 0.0 ? wl[k] : wr[k]);
    }
}

// explicit sources (curvature, gravity) of eq. `sources` at the cell centre
// (R, Z), iR = 1 / R, om2 = GM / r^3
__device__ inline void sources(const Prim &p, double R, double iR, double Z, double om2,
                               double S[4]) {
    S[0] = 0.0;
    S[1] = p.r * p.vp * p.vp * iR - p.r * (om2 * R);
    S[2] = 0.0;
    S[3] = -p.r * (om2 * Z);
}

// primitives of Q (iR = 1 / the radius of the angular momentum); empty cells at rest
__device__ inline Prim primitive(const double Q[4], double iR) {
    Prim p;
    p.r = Q[0];
    if (Q[0] >= DBL_MIN) {
        const double iq = 1.0 / Q[0];
        p.vR = Q[1] * iq;
        p.vp = Q[2] * iq * iR;
        p.vZ = Q[3] * iq;
    } else if (Q[0] > 0.0) {
        // a subnormal density (the coagulation update leaves such tails in
        // the upper bins): 1 / Q[0] would overflow, the quotients do not
        p.vR = Q[1] / Q[0];
        p.vp = Q[2] / Q[0] * iR;
        p.vZ = Q[3] / Q[0];
    } else {
        p.vR = p.vp = p.vZ = 0.0;
    }
    return p;
}

// Outward flux x area summed over the four faces of cell (i, j), species s,
// from states P (order 1: the cells' own values; order 2: piecewise linear)
// and the diffusive flux of eps = rho / rho_g between the cells.
template <int ORDER>
__device__ void flux_area(const TGeo &g, const GasT &gas, const double *rho, const double *v,
                          int i, int j, int s, double FA[4]) {
    const int nr = g.nr, nz = g.nz;
    const long c = (long)i * nz + j;
    // the cross stencil
    const Prim P0 = fetch(g, rho, v, i, j, s);
    const Prim Pw = fetch(g, rho, v, i - 1, j, s), Pe = fetch(g, rho, v, i + 1, j, s);
    const Prim Ps = fetch(g, rho, v, i, j - 1, s), Pn = fetch(g, rho, v, i, j + 1, s);
    Prim Lw = Pw, Rw = P0, Le = P0, Re = Pe;         // states at the west/east (R) faces
    Prim Ls = Ps, Rs = P0, Ln = P0, Rn = Pn;         // south/north (cone) faces
    if (ORDER == 2) {
        const Prim Pww = fetch(g, rho, v, i - 2, j, s), Pee = fetch(g, rho, v, i + 2, j, s);
        const Prim Pss = fetch(g, rho, v, i, j - 2, s), Pnn = fetch(g, rho, v, i, j + 2, s);
        const double *Rx = g.Rx + 2, *tx = g.tx + 2;     // index -2 .. n + 1
        const double *irx = g.irx + 2, *itx = g.itx + 2; // index -2 .. n
        const Prim gw = slope(Pww, Pw, P0, irx[i - 2], irx[i - 1]);
        const Prim g0 = slope(Pw, P0, Pe, irx[i - 1], irx[i]);
        const Prim ge = slope(P0, Pe, Pee, irx[i], irx[i + 1]);
        Lw = extrap(Pw, gw, g.Re[i] - Rx[i - 1]);
        Rw = extrap(P0, g0, g.Re[i] - Rx[i]);
        Le = extrap(P0, g0, g.Re[i + 1] - Rx[i]);
        Re = extrap(Pe, ge, g.Re[i + 1] - Rx[i + 1]);
        const Prim gs = slope(Pss, Ps, P0, itx[j - 2], itx[j - 1]);
        const Prim h0 = slope(Ps, P0, Pn, itx[j - 1], itx[j]);
        const Prim gn = slope(P0, Pn, Pnn, itx[j], itx[j + 1]);
        Ls = extrap(Ps, gs, g.te[j] - tx[j - 1]);
        Rs = extrap(P0, h0, g.te[j] - tx[j]);
        Ln = extrap(P0, h0, g.te[j + 1] - tx[j]);
        Rn = extrap(Pn, gn, g.te[j + 1] - tx[j + 1]);
    }
    // diffusion: -K (eps_r - eps_l), eps = rho / rho_g, K the face's
    // coefficient over the cells' distance (0 where the grid ends: the ghost
    // cells' eps, taken from the cells they copy, then carry no flux)
    const long kw = i > 0 ? c - nz : c, ke = i < nr - 1 ? c + nz : c;
    const long ks = j > 0 ? c - 1 : c, kn = j < nz - 1 ? c + 1 : c;
    const double e0 = P0.r * gas.irg[c];
    const double Fw = -gas.KR[c] * (e0 - Pw.r * gas.irg[kw]);
    const double Fe = -gas.KR[c + nz] * (Pe.r * gas.irg[ke] - e0);
    const long ft = (long)i * (nz + 1) + j;
    const double Fs = -gas.Kt[ft] * (e0 - Ps.r * gas.irg[ks]);
    const double Fn = -gas.Kt[ft + 1] * (Pn.r * gas.irg[kn] - e0);
    double fw[4], fe[4], fs[4], fn[4];
    face_flux(Lw, Rw, 1.0, 0.0, g.Re[i], Fw, fw);
    face_flux(Le, Re, 1.0, 0.0, g.Re[i + 1], Fe, fe);
    face_flux(Ls, Rs, g.nRt[j], g.nZt[j], g.Rcone[i], Fs, fs);
    face_flux(Ln, Rn, g.nRt[j + 1], g.nZt[j + 1], g.Rcone[i], Fn, fn);
    const double aw = g.AR[c], ae = g.AR[c + nz];
    const double as = g.At[ft], an = g.At[ft + 1];
#pragma unroll
    for (int k = 0; k < 4; ++k) FA[k] = ((0.0 - fw[k] * aw) + fe[k] * ae) - fs[k] * as + fn[k] * an;
}

// the tables of GasT from the gas arrays (one thread per cell)
__global__ __launch_bounds__(kTBlock) void k_tr_prep(TGeo g, Gas gas, double *irg, double *tsf,
                                                      double *KR, double *Kt) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nr = g.nr, nz = g.nz;
    if (c >= (long)nr * nz) return;
    const int i = (int)(c / nz), j = (int)(c - (long)i * nz);
    auto D = [&](long k) { return gas.rho_g[k] * (gas.alpha[k] * gas.c_s[k] * gas.H[k]) / g.Sc; };
    const double D0 = D(c);
    irg[c] = 1.0 / gas.rho_g[c];
    tsf[c] = g.rho_m / (gas.rho_g[c] * (sqrt(8.0 / M_PI) * gas.c_s[c]));
    KR[c] = i > 0 ? 0.5 * (D(c - nz) + D0) / (g.Rc[i] - g.Rc[i - 1]) : 0.0;
    if (i == nr - 1) KR[c + nz] = 0.0;
    const long ft = (long)i * (nz + 1) + j;
    Kt[ft] = j > 0 ? 0.5 * (D(c - 1) + D0) / (g.nZt[j] * g.Rc[i] * (g.tc[j] - g.tc[j - 1])) : 0.0;
    if (j == nz - 1) Kt[ft + 1] = 0.0;
}

// Each wave takes the species of one cell (lane = species within a run of
// 64): the cell's index, and so every gas and geometry operand, is uniform
// over the wave and read through the scalar cache; only the states of the
// stencil are vector loads.  The waves of a cell are ceil(N / 64) in a row.
__device__ inline bool wave_cell(const TGeo &g, long &c, int &s) {
    const int wpc = (g.N + 63) >> 6;                 // waves per cell
    const long w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kTBlock / 64) + (threadIdx.x >> 6)));
    c = w / wpc;
    s = (int)(w - c * wpc) * 64 + (int)(threadIdx.x & 63);
    return c < (long)g.nr * g.nz && s < g.N;
}

// Stages (i)-(iv): first-order fluxes at t^n, half update, half source,
// primitives, half drag -> the half-step state (rh, vh)
__global__ __launch_bounds__(kTBlock) void k_tr_half(TGeo g, GasT gas, const double *rho,
                                                      const double *v, double *rh, double *vh,
                                                      double dt) {
    long c;
    int s;
    if (!wave_cell(g, c, s)) return;
    const long t = c * g.N + s;
    const int i = (int)(c / g.nz), j = (int)(c - (long)i * g.nz);
    double FA[4];
    flux_area<1>(g, gas, rho, v, i, j, s, FA);
    const double R = g.Rc[i], iR = g.iRc[i], Z = g.tc[j] * g.Rc[i];
    const Prim P = {rho[t], v[3 * t], v[3 * t + 1], v[3 * t + 2]};
    const double Q[4] = {P.r, P.r * P.vR, P.r * P.vp * R, P.r * P.vZ};
    double S[4];
    sources(P, R, iR, Z, g.om2[c], S);
    const double f = 0.5 * dt * g.iV[c];
    double Qs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) Qs[k] = (Q[k] - f * FA[k]) + 0.5 * dt * S[k];
    Prim H = primitive(Qs, iR);
    const double hd = 0.5 * dt, w = hd / (hd + gas.tsf[c] * g.s[s]);
    const double *vg = gas.v_g + 3 * c;
    // below the floor the species moves with the gas
    const bool fl = g.eps_floor > 0.0 && H.r < g.eps_floor * gas.rho_g[c];
    rh[t] = H.r;
    vh[3 * t] = fl ? vg[0] : H.vR - w * (H.vR - vg[0]);
    vh[3 * t + 1] = fl ? vg[1] : H.vp - w * (H.vp - vg[1]);
    vh[3 * t + 2] = fl ? vg[2] : H.vZ - w * (H.vZ - vg[2]);
}

// Stages (v)-(viii): second-order fluxes at t^{n+1/2}, full update from t^n,
// full source at t^{n+1/2}, primitives, full drag, in place on (rho, v)
// (a thread reads only its own cell's t^n state)
__global__ __launch_bounds__(kTBlock) void k_tr_full(TGeo g, GasT gas, double *rho, double *v,
                                                      const double *rh, const double *vh,
                                                      double dt) {
    long c;
    int s;
    if (!wave_cell(g, c, s)) return;
    const long t = c * g.N + s;
    const int i = (int)(c / g.nz), j = (int)(c - (long)i * g.nz);
    double FA[4];
    flux_area<2>(g, gas, rh, vh, i, j, s, FA);
    const double R = g.Rc[i], iR = g.iRc[i], Z = g.tc[j] * g.Rc[i];
    const Prim P = {rho[t], v[3 * t], v[3 * t + 1], v[3 * t + 2]};
    const double Q[4] = {P.r, P.r * P.vR, P.r * P.vp * R, P.r * P.vZ};
    const Prim Ph = {rh[t], vh[3 * t], vh[3 * t + 1], vh[3 * t + 2]};
    double S[4];
    sources(Ph, R, iR, Z, g.om2[c], S);
    const double f = dt * g.iV[c];
    double Qd[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) Qd[k] = (Q[k] - f * FA[k]) + dt * S[k];
    const Prim N1 = primitive(Qd, iR);
    const double w = dt / (dt + gas.tsf[c] * g.s[s]);
    const double *vg = gas.v_g + 3 * c;
    const bool fl = g.eps_floor > 0.0 && N1.r < g.eps_floor * gas.rho_g[c];
    rho[t] = N1.r;
    v[3 * t] = fl ? vg[0] : N1.vR - w * (N1.vR - vg[0]);
    v[3 * t + 1] = fl ? vg[1] : N1.vp - w * (N1.vp - vg[1]);
    v[3 * t + 2] = fl ? vg[2] : N1.vZ - w * (N1.vZ - vg[2]);
}

// positive doubles order like their bit patterns: the minimum via atomicMin on them
__global__ void k_tr_fill(unsigned long long *x, unsigned long long val) { *x = val; }

// each block strides over the (cell, species) pairs and adds one atomic: a
// bounded grid keeps the atomics on the one word few
constexpr int kCflBlocks = 1024;

__global__ __launch_bounds__(kTBlock) void k_tr_cfl(TGeo g, Gas gas, const double *v,
                                                     double c_adv, double c_diff,
                                                     unsigned long long *out) {
    __shared__ double red[kTBlock / 64];
    const long C = (long)g.nr * g.nz;
    double m = INFINITY;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < C * g.N;
         t += (long)gridDim.x * blockDim.x) {
        const long c = t / g.N;
        const int i = (int)(c / g.nz), j = (int)(c - (long)i * g.nz);
        const double dR = g.dR[i], dZ = g.Rc[i] * (g.te[j + 1] - g.te[j]);
        const double a = fmin(fabs(dR / v[3 * t]), fabs(dZ / v[3 * t + 2]));
        const double k = gas.alpha[c] * gas.c_s[c] * gas.H[c] / g.Sc;
        const double d = fmin(dR * dR / k, dZ * dZ / k);
        m = fmin(m, fmin(c_adv * a, c_diff * d));
    }
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int w = 1; w < kTBlock / 64; ++w) b = fmin(b, red[w]);
        if (b < INFINITY) atomicMin(out, (unsigned long long)__double_as_longlong(b));
    }
}

// smallest h and number of non-zero statuses over C cells (the scheduler's trigger)
__global__ __launch_bounds__(kTBlock) void k_tr_trigger(const double *h, const int32_t *status,
                                                         long C, unsigned long long *hmin,
                                                         int *nbad) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double m = INFINITY;
    int bad = 0;
    if (t < C) {
        m = h[t] > 0.0 ? h[t] : INFINITY;
        bad = status ? (status[t] != 0) : 0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        m = fmin(m, __shfl_xor(m, o, 64));
        bad += __shfl_xor(bad, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (m < INFINITY) atomicMin(hmin, (unsigned long long)__double_as_longlong(m));
        if (bad) atomicAdd(nbad, bad);
    }
}

}  // namespace
}  // namespace coag

using namespace coag;

struct coag_tctx {
    int nr = 0, nz = 0, N = 0;
    double GM = 0, Sc = 1, c_adv = 0.4, c_diff = 0.2, rho_m = 0;
    double *tables = nullptr;             // all geometry arrays in one allocation
    TGeo geo{};
    double *rh = nullptr, *vh = nullptr;  // half-step state
    double *gt = nullptr;                 // gas tables (GasT), refreshed by every step
    unsigned long long *red = nullptr;    // reduction scalars (dt, hmin) and a counter
    // scheduler workspace
    void *K = nullptr;
    size_t K_bytes = 0;
    int32_t *nsub = nullptr, *status = nullptr;
    long ws_cells = 0;
    std::string err;
};

namespace {
thread_local std::string g_terr;

int tfail(coag_tctx *t, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    (t ? t->err : g_terr) = buf;
    return code;
}

#define THIP(t, call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return tfail(t, COAG_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

Gas gas_of(const coag_cells *cells, const double *v_gas) {
    return Gas{cells->rho_g, cells->c_s, cells->H, cells->alpha, v_gas};
}

bool cells_ok(const coag_cells *c) {
    return c && c->rho_g && c->c_s && c->H && c->alpha;
}
}  // namespace

extern "C" {

int coag_transport_create(const coag_tgrid *grid, int32_t N, const double *s, double rho_m,
                          coag_tctx **out) {
    if (!out) return tfail(nullptr, COAG_EINVAL, "coag_transport_create: out is NULL");
    *out = nullptr;
    if (!grid || !grid->R_edge || !grid->t_edge || !s)
        return tfail(nullptr, COAG_EINVAL, "coag_transport_create: NULL grid, edges or radii");
    const int nr = grid->n_r, nz = grid->n_z;
    if (nr < 1 || nz < 1 || N < 1 || N > 1023)
        return tfail(nullptr, COAG_EINVAL, "coag_transport_create: n_r = %d, n_z = %d, N = %d", nr,
                     nz, N);
    if (!(rho_m > 0.0) || !(grid->Sc > 0.0) || !(grid->c_adv > 0.0) || !(grid->c_diff > 0.0) ||
        !(grid->GM >= 0.0) || !(grid->eps_floor >= 0.0) || !std::isfinite(grid->eps_floor))
        return tfail(nullptr, COAG_EINVAL,
                     "coag_transport_create: need rho_m, Sc, c_adv, c_diff > 0, GM >= 0 and a "
                     "finite eps_floor >= 0");
    const double *Re = grid->R_edge, *te = grid->t_edge;
    if (!(Re[0] > 0.0) || te[0] != 0.0)
        return tfail(nullptr, COAG_EINVAL, "coag_transport_create: need R_edge[0] > 0, t_edge[0] = 0");
    for (int i = 0; i < nr; ++i)
        if (!(Re[i + 1] > Re[i]))
            return tfail(nullptr, COAG_EINVAL, "coag_transport_create: R_edge not increasing at %d", i);
    for (int j = 0; j < nz; ++j)
        if (!(te[j + 1] > te[j]))
            return tfail(nullptr, COAG_EINVAL, "coag_transport_create: t_edge not increasing at %d", j);
    for (int k = 0; k < N; ++k)
        if (!(s[k] > 0.0)) return tfail(nullptr, COAG_EINVAL, "coag_transport_create: s[%d] <= 0", k);

    // host geometry: every table in one array, in this order
    const long nRc = nr, nRe = nr + 1, ndR = nr, nRcone = nr, nRx = nr + 4, ntc = nz, nte = nz + 1,
               ntx = nz + 4, nV = (long)nr * nz, nAR = (long)(nr + 1) * nz,
               nAt = (long)nr * (nz + 1), ns = N, nirx = nr + 3, nitx = nz + 3, nnt = nz + 1;
    std::vector<double> h(nRc + nRe + ndR + nRcone + nRx + ntc + nte + ntx + nV + nAR + nAt + ns +
                          nRc + nirx + nitx + 2 * nnt + 2 * nV);
    double *p = h.data();
    double *Rc = p; p += nRc;
    double *Rev = p; p += nRe;
    double *dR = p; p += ndR;
    double *Rcone = p; p += nRcone;
    double *Rx = p; p += nRx;
    double *tc = p; p += ntc;
    double *tev = p; p += nte;
    double *tx = p; p += ntx;
    double *V = p; p += nV;
    double *AR = p; p += nAR;
    double *At = p; p += nAt;
    double *sv = p; p += ns;
    double *iRc = p; p += nRc;
    double *irx = p; p += nirx;
    double *itx = p; p += nitx;
    double *nRt = p; p += nnt;
    double *nZt = p; p += nnt;
    double *iV = p; p += nV;
    double *om2 = p;
    for (int i = 0; i <= nr; ++i) Rev[i] = Re[i];
    for (int j = 0; j <= nz; ++j) tev[j] = te[j];
    for (int i = 0; i < nr; ++i) {
        const double a = Re[i], b = Re[i + 1];
        Rc[i] = sqrt(a * b);
        dR[i] = b - a;
        Rcone[i] = (2.0 / 3.0) * (b * b * b - a * a * a) / (b * b - a * a);
    }
    for (int j = 0; j < nz; ++j) tc[j] = 0.5 * (te[j] + te[j + 1]);
    // ghost coordinates: mirrored about the edge faces (the second ghost about
    // the edge too, from the second cell; one extra width when there is none)
    Rx[2 + 0 - 1] = 2.0 * Re[0] - Rc[0];
    Rx[2 + 0 - 2] = nr > 1 ? 2.0 * Re[0] - Rc[1] : 2.0 * Re[0] - Rc[0] - (Re[1] - Re[0]);
    for (int i = 0; i < nr; ++i) Rx[2 + i] = Rc[i];
    Rx[2 + nr] = 2.0 * Re[nr] - Rc[nr - 1];
    Rx[2 + nr + 1] = nr > 1 ? 2.0 * Re[nr] - Rc[nr - 2] : Rx[2 + nr] + (Re[1] - Re[0]);
    tx[1] = -tc[0];
    tx[0] = nz > 1 ? -tc[1] : -tc[0] - (te[1] - te[0]);
    for (int j = 0; j < nz; ++j) tx[2 + j] = tc[j];
    tx[2 + nz] = 2.0 * te[nz] - tc[nz - 1];
    tx[2 + nz + 1] = nz > 1 ? 2.0 * te[nz] - tc[nz - 2] : tx[2 + nz] + (te[1] - te[0]);
    for (int i = 0; i < nr; ++i) {
        const double a = Re[i], b = Re[i + 1];
        for (int j = 0; j < nz; ++j)
            V[(long)i * nz + j] = (2.0 * M_PI / 3.0) * (b * b * b - a * a * a) * (te[j + 1] - te[j]);
        for (int j = 0; j <= nz; ++j)
            At[(long)i * (nz + 1) + j] = M_PI * (b * b - a * a) * sqrt(1.0 + te[j] * te[j]);
    }
    for (int i = 0; i <= nr; ++i)
        for (int j = 0; j < nz; ++j) AR[(long)i * nz + j] = 2.0 * M_PI * Re[i] * Re[i] * (te[j + 1] - te[j]);
    for (int k = 0; k < N; ++k) sv[k] = s[k];
    // reciprocals and normals the kernels would otherwise divide for per thread
    for (int i = 0; i < nr; ++i) iRc[i] = 1.0 / Rc[i];
    for (int k = 0; k < nirx; ++k) irx[k] = 1.0 / (Rx[k + 1] - Rx[k]);
    for (int k = 0; k < nitx; ++k) itx[k] = 1.0 / (tx[k + 1] - tx[k]);
    for (int j = 0; j <= nz; ++j) {
        const double cj = 1.0 / sqrt(1.0 + te[j] * te[j]);
        nRt[j] = -te[j] * cj;
        nZt[j] = cj;
    }
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nz; ++j) {
            const long c = (long)i * nz + j;
            const double R = Rc[i], Z = tc[j] * Rc[i], r2 = R * R + Z * Z;
            iV[c] = 1.0 / V[c];
            om2[c] = grid->GM / (r2 * sqrt(r2));
        }

    coag_tctx *t = new coag_tctx();
    t->nr = nr;
    t->nz = nz;
    t->N = N;
    t->GM = grid->GM;
    t->Sc = grid->Sc;
    t->c_adv = grid->c_adv;
    t->c_diff = grid->c_diff;
    t->rho_m = rho_m;
    const long C = (long)nr * nz;
    if (hipMalloc(&t->tables, h.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&t->rh, (size_t)C * N * 4 * sizeof(double)) != hipSuccess ||
        hipMalloc(&t->gt, (size_t)(2 * C + nAR + nAt) * sizeof(double)) != hipSuccess ||
        hipMalloc(&t->red, 4 * sizeof(unsigned long long)) != hipSuccess) {
        coag_transport_destroy(t);
        return tfail(nullptr, COAG_ENOMEM, "coag_transport_create: device allocation failed");
    }
    t->vh = t->rh + (size_t)C * N;
    if (hipMemcpy(t->tables, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        coag_transport_destroy(t);
        return tfail(nullptr, COAG_EHIP, "coag_transport_create: copy of the geometry failed");
    }
    double *d = t->tables;
    TGeo &g = t->geo;
    g.nr = nr;
    g.nz = nz;
    g.N = N;
    g.Rc = d; d += nRc;
    g.Re = d; d += nRe;
    g.dR = d; d += ndR;
    g.Rcone = d; d += nRcone;
    g.Rx = d; d += nRx;
    g.tc = d; d += ntc;
    g.te = d; d += nte;
    g.tx = d; d += ntx;
    g.V = d; d += nV;
    g.AR = d; d += nAR;
    g.At = d; d += nAt;
    g.s = d; d += ns;
    g.iRc = d; d += nRc;
    g.irx = d; d += nirx;
    g.itx = d; d += nitx;
    g.nRt = d; d += nnt;
    g.nZt = d; d += nnt;
    g.iV = d; d += nV;
    g.om2 = d;
    g.rho_m = rho_m;
    g.GM = grid->GM;
    g.Sc = grid->Sc;
    g.eps_floor = grid->eps_floor;
    *out = t;
    return COAG_OK;
}

void coag_transport_destroy(coag_tctx *t) {
    if (!t) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(t->tables);
    (void)hipFree(t->rh);
    (void)hipFree(t->gt);
    (void)hipFree(t->red);
    (void)hipFree(t->K);
    (void)hipFree(t->nsub);
    delete t;
}

const char *coag_transport_last_error(const coag_tctx *t) { return t ? t->err.c_str() : g_terr.c_str(); }

int coag_transport_dt(coag_tctx *t, const coag_cells *cells, const double *v, double *dt_out,
                      void *stream) {
    if (!t) return tfail(nullptr, COAG_EINVAL, "coag_transport_dt: t is NULL");
    if (!cells_ok(cells) || !v || !dt_out)
        return tfail(t, COAG_EINVAL, "coag_transport_dt: NULL cells, v or dt_out");
    hipStream_t st = (hipStream_t)stream;
    const long n = (long)t->nr * t->nz * t->N;
    hipLaunchKernelGGL(k_tr_fill, dim3(1), dim3(1), 0, st, t->red, 0x7FF0000000000000ull);
    const long nb = std::min<long>((n + kTBlock - 1) / kTBlock, kCflBlocks);
    hipLaunchKernelGGL(k_tr_cfl, dim3((unsigned)std::max<long>(nb, 1)), dim3(kTBlock), 0, st,
                       t->geo, gas_of(cells, nullptr), v, t->c_adv, t->c_diff, t->red);
    THIP(t, hipGetLastError());
    unsigned long long bits = 0;
    THIP(t, hipMemcpyAsync(&bits, t->red, sizeof bits, hipMemcpyDeviceToHost, st));
    THIP(t, hipStreamSynchronize(st));
    double dt;
    memcpy(&dt, &bits, sizeof dt);
    *dt_out = dt;
    return COAG_OK;
}

int coag_transport_step(coag_tctx *t, const coag_cells *cells, const double *v_gas, double *rho,
                        double *v, double dt, void *stream) {
    if (!t) return tfail(nullptr, COAG_EINVAL, "coag_transport_step: t is NULL");
    if (!cells_ok(cells) || !v_gas || !rho || !v)
        return tfail(t, COAG_EINVAL, "coag_transport_step: NULL cells, v_gas, rho or v");
    if (!(dt > 0.0) || !std::isfinite(dt))
        return tfail(t, COAG_EINVAL, "coag_transport_step: dt = %g", dt);
    hipStream_t st = (hipStream_t)stream;
    const long waves = (long)t->nr * t->nz * ((t->N + 63) / 64);
    const dim3 grid((unsigned)((waves + kTBlock / 64 - 1) / (kTBlock / 64)));
    const long C = (long)t->nr * t->nz;
    double *irg = t->gt, *tsf = irg + C, *KR = tsf + C, *Kt = KR + (long)(t->nr + 1) * t->nz;
    hipLaunchKernelGGL(k_tr_prep, dim3((unsigned)((C + kTBlock - 1) / kTBlock)), dim3(kTBlock), 0,
                       st, t->geo, gas_of(cells, v_gas), irg, tsf, KR, Kt);
    const GasT gas{irg, tsf, KR, Kt, v_gas, cells->rho_g};
    hipLaunchKernelGGL(k_tr_half, grid, dim3(kTBlock), 0, st, t->geo, gas, rho, v, t->rh, t->vh, dt);
    hipLaunchKernelGGL(k_tr_full, grid, dim3(kTBlock), 0, st, t->geo, gas, rho, v, t->rh, t->vh, dt);
    THIP(t, hipGetLastError());
    return COAG_OK;
}

int coag_evolve(coag_ctx *ctx, coag_tctx *t, int64_t C, const coag_cells *cells,
                const double *v_gas, const double *v_frag, double *rho, double *v, double *h,
                double t_end, int64_t max_steps, const coag_tol *tol, coag_evolve_stats *stats,
                void *stream) {
    if (!t) return tfail(nullptr, COAG_EINVAL, "coag_evolve: t is NULL");
    if (!ctx || !cells_ok(cells) || !v_gas || !v_frag || !rho || !v || !h || !tol)
        return tfail(t, COAG_EINVAL, "coag_evolve: NULL argument");
    if (C != (int64_t)t->nr * t->nz)
        return tfail(t, COAG_EINVAL, "coag_evolve: C = %lld, the grid has %lld cells", (long long)C,
                     (long long)t->nr * t->nz);
    if (ctx_bins(ctx) != t->N)
        return tfail(t, COAG_EINVAL, "coag_evolve: %d bins in the coagulation context, %d species",
                     ctx_bins(ctx), t->N);
    if (ctx_vertical(ctx))
        return tfail(t, COAG_EINVAL,
                     "coag_evolve: the transport carries volume densities; the coagulation "
                     "context takes the vertically integrated kernel's surface densities");
    if (!(t_end > 0.0) || !std::isfinite(t_end) || max_steps < 1)
        return tfail(t, COAG_EINVAL, "coag_evolve: t_end = %g, max_steps = %lld", t_end,
                     (long long)max_steps);
    if (tol->mode != COAG_ADAPTIVE || (tol->prec != COAG_PREC_FP64 && tol->prec != COAG_PREC_SPLIT_BF16))
        return tfail(t, COAG_EINVAL, "coag_evolve: needs ADAPTIVE steps in FP64 or split precision");
    hipStream_t st = (hipStream_t)stream;
    const int N = t->N;
    const bool split = tol->prec == COAG_PREC_SPLIT_BF16;
    // blocked rates where the batched step applies; otherwise (FP64 only) the
    // per-cell step with [C][P] rates
    const bool blocked = ctx_blocked(ctx, split ? 1 : 0);
    if (split && !blocked)
        return tfail(t, COAG_ENOTSUP,
                     "coag_evolve: split precision needs the batched step, which this "
                     "context's grid does not allow (N >= 16 bins whose products of each row "
                     "fit a 16-bin window)");
    const long m = N >> 1;
    const long SL = (N & 1) ? (m + 1) * (m + 1) : m * (m + 1);
    const long P = (long)N * (N + 1) / 2;
    const size_t kb = blocked ? (size_t)64 * SL * ((C + 15) / 16) * (split ? 4 : 8)
                              : (size_t)2 * C * P * sizeof(double);
    if (kb > t->K_bytes) {
        (void)hipFree(t->K);
        t->K = nullptr;
        t->K_bytes = 0;
        if (hipMalloc(&t->K, kb) != hipSuccess) return tfail(t, COAG_ENOMEM, "coag_evolve: rates");
        t->K_bytes = kb;
    }
    if (C > t->ws_cells) {
        (void)hipFree(t->nsub);
        t->nsub = nullptr;
        t->ws_cells = 0;
        if (hipMalloc(&t->nsub, (size_t)C * 2 * sizeof(int32_t)) != hipSuccess)
            return tfail(t, COAG_ENOMEM, "coag_evolve: step counters");
        t->status = t->nsub + C;
        t->ws_cells = C;
    }
    coag_tol tl = *tol;
    tl.rates_layout = !blocked ? COAG_RATES_CP64 : split ? COAG_RATES_BLK32 : COAG_RATES_BLK64;
    const dim3 cg((unsigned)((C + kTBlock - 1) / kTBlock));
    // the trigger: smallest positive h of the cells (0 if none), and the failed cells
    auto trigger = [&](double &hmin, int &nbad, bool with_status) -> int {
        hipLaunchKernelGGL(k_tr_fill, dim3(1), dim3(1), 0, st, t->red + 1, 0x7FF0000000000000ull);
        hipLaunchKernelGGL(k_tr_fill, dim3(1), dim3(1), 0, st, t->red + 2, 0ull);
        hipLaunchKernelGGL(k_tr_trigger, cg, dim3(kTBlock), 0, st, h,
                           with_status ? t->status : (const int32_t *)nullptr, (long)C, t->red + 1,
                           (int *)(t->red + 2));
        THIP(t, hipGetLastError());
        unsigned long long r[2];
        THIP(t, hipMemcpyAsync(r, t->red + 1, sizeof r, hipMemcpyDeviceToHost, st));
        THIP(t, hipStreamSynchronize(st));
        double x;
        memcpy(&x, &r[0], sizeof x);
        hmin = x < INFINITY ? x : 0.0;
        nbad = (int)(r[1] & 0xffffffffu);
        return COAG_OK;
    };
    double trig = 0.0;
    int nbad = 0;
    int rc = trigger(trig, nbad, false);
    if (rc) return rc;
    nbad = 0;
    double time = 0.0, since = 0.0;
    int64_t steps = 0, calls = 0;
    while (time < t_end) {
        if (steps >= max_steps) {
            if (stats) *stats = coag_evolve_stats{steps, calls, time, nbad};
            return tfail(t, COAG_EINVAL, "coag_evolve: %lld transport steps reached before t_end",
                         (long long)max_steps);
        }
        double dt;
        rc = coag_transport_dt(t, cells, v, &dt, stream);
        if (rc) return rc;
        const bool last = !(dt < t_end - time);
        if (last) dt = t_end - time;
        rc = coag_transport_step(t, cells, v_gas, rho, v, dt, stream);
        if (rc) return rc;
        ++steps;
        time = last ? t_end : time + dt;
        since += dt;
        if (since >= trig || last) {
            double *Kc = (double *)t->K, *Kf = blocked ? nullptr : Kc + C * P;
            rc = blocked ? coag_rates_blocked(ctx, C, cells, v, v_frag, split ? 1 : 0, t->K, stream)
                         : coag_rates(ctx, C, cells, v, v_frag, Kc, Kf, stream);
            if (rc) return tfail(t, rc, "coag_evolve: rates: %s", coag_last_error(ctx));
            rc = coag_step(ctx, C, rho, t->K, Kf, since, h, &tl, t->nsub, nullptr, nullptr,
                           t->status, stream);
            if (rc) return tfail(t, rc, "coag_evolve: step: %s", coag_last_error(ctx));
            ++calls;
            since = 0.0;
            rc = trigger(trig, nbad, true);
            if (rc) return rc;
        }
    }
    if (stats) *stats = coag_evolve_stats{steps, calls, time, nbad};
    return COAG_OK;
}

}  // extern "C"
