// coag_rate.h -- the pair-rate arithmetic (Sec. 5, eqs. `kernel`, `vbrown`,
// `OCVrel`, `p_frag`, `t_stop`) of the rate kernels (coag_kernels.hip): the
// per-cell and per-grain terms, one pair's rates, and the writer of one
// 16-cell block in the blocked layout.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "coag_device.h"
#include "coag_launch.h"

namespace coag {

// ---------------------------------------------------------------------------
// Pair rates.  Everything in the Ormel & Cuzzi expressions that depends on one
// bin only is tabulated per cell in LDS first.  Stokes numbers grow
// with grain size, so the heavier grain i of a pair is the one with the larger
// Stokes number: St_1 = St_i, St* = clamp(y* St_i, Re^-1/2, 1) is a per-row
// value, and per pair only (St_i - St_j) / (St_i + St_j) and
// St_j^2 / (St* + St_j) remain to divide (plus v_frag / dv).
//   A_k = St_k^2 / (1 + St_k),  B_k = St_k^2 / (St_k + delta),
//   S_k = clamp(y* St_k, delta, 1),  C_k = St_k^2 / (S_k + St_k)
//   dV_I^2  = (St_i - St_j)/(St_i + St_j) (C_i - A_i - q + A_j)
//   dV_II^2 = 2 (S_i - delta) + C_i - B_i + q - B_j,   q = St_j^2 / (S_i + St_j)
// ---------------------------------------------------------------------------
// Constants of one cell (H2 = H^2 and alpha for the vertically integrated
// kernel's scale heights).
struct CellRate {
    double delta, vt_scale, kbt, vf, rg_vth, Om, H2, alpha;
    bool turb;
};

__device__ inline CellRate cell_rate(const CellArrays &cells, const double *v_frag, long c) {
    CellRate r;
    const double c_s = cells.c_s[c], alpha = cells.alpha[c];
    r.H2 = cells.H[c] * cells.H[c];
    r.alpha = alpha;
    r.turb = alpha > 0.0;
    r.delta = r.turb ? 1.0 / sqrt(alpha * c_s * cells.H[c] / cells.nu_mol[c]) : 0.0;
    r.vt_scale = alpha * c_s * c_s;
    r.kbt = 8.0 * kBoltzmann * cells.T[c] / M_PI;
    r.vf = v_frag[c];
    r.rg_vth = cells.rho_g[c] * (sqrt(8.0 / M_PI) * c_s);      // rho_g v_th
    r.Om = cells.Omega[c];
    return r;
}

// One grain of one cell: St, A, B, C above, velocity, 1/m, radius, the
// squared scale height h^2 (vertically integrated kernel); and, for the
// heavier grain of a pair, S, u = C - A and w = 2 (S - delta) + C - B.
struct Grain {
    double st, a, bt, ct, vx, vy, vz, im, s, h2;
    double S, u, w;
};

// Vertically integrated kernel (Sec. 5.1): a grain's column has a Gaussian
// vertical profile of scale height h = H sqrt(alpha / (alpha + St)) (mixing
// against settling), and its vertical velocity is the terminal settling
// speed St Omega Z at Z = h.  The pair rate is the volume rate integrated
// over height: K / sqrt(2 pi (h_i^2 + h_j^2)).  Needs alpha > 0 (h = 0
// otherwise, and the rates are not finite).
__device__ inline double grain_h2(const CellRate &r, double st) {
    return r.H2 * (r.alpha / (r.alpha + st));
}
__device__ inline double settle_speed(const CellRate &r, double st, double h2) {
    return st * r.Om * sqrt(h2);
}

__device__ inline double stir_s(const CellRate &r, double st) {
    return fmin(fmax(kYStar * st, r.delta), 1.0);
}

// A, B, C of a grain of Stokes number st
__device__ inline void grain_abc(const CellRate &r, double st, Grain &g) {
    const double a = st * st;
    g.st = st;
    g.a = a / (1.0 + st);
    g.bt = r.turb ? a / (st + r.delta) : 0.0;
    g.ct = a / (stir_s(r, st) + st);
}

// St, A, B, C of a grain of radius s (material density rho_m)
__device__ inline void grain_terms(const CellRate &r, double rho_m, double s, Grain &g) {
    grain_abc(r, rho_m * s / r.rg_vth * r.Om, g);
}

// the heavier grain's S, u, w (S given)
__device__ inline void heavier_terms(const CellRate &r, Grain &g, double S) {
    g.S = S;
    g.u = g.ct - g.a;
    g.w = 2.0 * (S - r.delta) + g.ct - g.bt;
}

// a / b and 1 / sqrt(x) for the per-pair arithmetic, whose operands are
// normal, finite and positive: the hardware estimates refined by Newton's
// iteration (reciprocal: r <- r + r (1 - b r), twice, then the quotient
// corrected once, q <- q + r (a - b q); reciprocal square root:
// r <- r (3/2 - x r^2 / 2), twice).  Within an ulp or two of the rounded
// results, in fewer instructions than the IEEE sequences, which also scale
// for denormal and overflowing operands.
// exp(-y) rounds to zero in FP64 for y above about 745.13
constexpr double kExpZeroY = 746.0;

__device__ __forceinline__ double div_nr(double a, double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    r = fma(fma(-b, r, 1.0), r, r);
    const double q = a * r;
    return fma(fma(-b, q, a), r, q);
}

__device__ __forceinline__ double rsqrt_nr(double x) {
    double r = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    r = r * fma(-hx * r, r, 1.5);
    r = r * fma(-hx * r, r, 1.5);
    return r;
}

// Kc, Kf of the pair (i, j), i >= j (i the grain with the larger St; its
// heavier_terms set); vertical: the vertically integrated kernel (the
// grains' vz are then their settling speeds, h2 their squared scale heights)
__device__ inline void pair_rates(const CellRate &r, const Grain &gi, const Grain &gj, bool diag,
                                  bool vertical, double &kc, double &kf) {
    double vturb2 = 0.0;
    if (r.turb) {
        const double si = gi.st, sj = gj.st;
        const double q = div_nr(sj * sj, gi.S + sj);
        const double dV1 = div_nr(si - sj, si + sj) * (gi.u - q + gj.a);
        const double dV2 = gi.w + q - gj.bt;
        vturb2 = r.vt_scale * (dV1 + dV2);
    }
    const double dx = gi.vx - gj.vx, dy = gi.vy - gj.vy, dz = gi.vz - gj.vz;
    // dv = sqrt(dv2) = dv2 / sqrt(dv2), and y = 1.5 (v_frag / dv)^2 = 1.5 v_frag^2 / dv2;
    // where dv2 > 0 fails (dv2 = 0, or NaN), dv = dv2 * 0 is 0 or NaN, as its
    // square root would be, without evaluating one
    const double dv2 = r.kbt * (gi.im + gj.im) + vturb2 + (dx * dx + dy * dy + dz * dz);
    const double rs = dv2 > 0.0 ? rsqrt_nr(dv2) : 0.0;
    const double dv = dv2 * rs;
    const double ss = gi.s + gj.s;
    double K = M_PI * ss * ss * dv * (diag ? 0.5 : 1.0);
    if (vertical) K *= rsqrt_nr(2.0 * M_PI * (gi.h2 + gj.h2));
    // past y = kExpZeroY, exp(-y) is zero in FP64 (denormals included), so
    // pf = 0 and pc = 1 exactly; pairs of slowly colliding grains, the most
    // common, then skip the exponential (a branch whole waves take together)
    double pf = 0.0, pc = 1.0;
    const double qv = r.vf * rs;
    const double y = 1.5 * qv * qv;
    if (dv2 > 0.0 && y < kExpZeroY) {
        pf = (1.0 + y) * exp(-y);
        pc = y < kSeriesY
                 ? y * y * (1.0 / 2.0 + y * (-1.0 / 3.0 + y * (1.0 / 8.0 + y * (-1.0 / 30.0 +
                   y * (1.0 / 144.0 + y * (-1.0 / 840.0 + y * (1.0 / 5760.0)))))))
                 : 1.0 - pf;
    }
    kc = K * pc;
    kf = K * pf;
}

// What the adjoint needs of one pair's rate derivatives with respect to the
// cell's alpha and v_frag (i >= j, so St_i >= St_j; plain FP64 divisions and
// square root).  alpha enters through v_turb^2 = alpha c_s^2 V(delta, S) with
// delta = Re^(-1/2) proportional to alpha^(-1/2) and S = clamp(y* St_i,
// delta, 1), which moves with delta only while it sits on the lower clamp:
//   d v_turb^2 / d alpha = c_s^2 (V - delta/2 dV/ddelta),
// and Z = (d dv / d alpha) / dv = (d v_turb^2 / d alpha) / (2 dv^2).
// v_frag enters through y = 1.5 (v_frag / dv)^2 in p_frag = (1 + y) e^-y.
// With X = 2 y^2 / (1 + y), the derivatives follow from the rates themselves
// (Kc = w K p_coag, Kf = w K p_frag, K = sigma dv):
//   dKc/dalpha = Z (Kc - X Kf),   dKf/dalpha = Z (1 + X) Kf,
//   dKf/dv_frag = -X Kf / v_frag = -dKc/dv_frag.
// With alpha = 0 the turbulent term is off and Z = 0; with dv = 0, or where
// e^-y is zero in FP64 (Kf = 0 there), X = 0.
//
// Vertically integrated kernel: alpha also moves the scale heights, with
// d ln h_k / d alpha = St_k / (2 alpha (alpha + St_k)) = e_k, hence the
// settling speeds (d vlam^2 / d alpha, passed in as dvlam2_da, joins
// d v_turb^2 / d alpha in Z) and the overlap factor G = (2 pi (h_i^2 +
// h_j^2))^(-1/2), whose W = d ln G / d alpha = -(h_i^2 e_i + h_j^2 e_j) /
// (h_i^2 + h_j^2) adds W Kc, W Kf to the two alpha derivatives (vertical_w).
struct RateDerivs {
    double Z, X;
};

__device__ inline double vertical_e(const CellRate &r, double st) {
    return st / (2.0 * r.alpha * (r.alpha + st));
}

__device__ inline double vertical_w(double h2_i, double e_i, double h2_j, double e_j) {
    return -(h2_i * e_i + h2_j * e_j) / (h2_i + h2_j);
}

__device__ inline RateDerivs pair_rate_derivs(const CellRate &r, double alpha, double cs2,
                                              double st_i, double st_j, double im_i,
                                              double im_j, double vlam2, double dvlam2_da) {
    double vturb2 = 0.0, dvt2_da = 0.0;
    if (r.turb) {
        const double d = r.delta;
        double S = kYStar * st_i, dS = 0.0;
        if (S < d) { S = d; dS = 1.0; }
        if (S > 1.0) { S = 1.0; dS = 0.0; }
        const double a1 = st_i * st_i, a2 = st_j * st_j, f12 = (st_i - st_j) / (st_i + st_j);
        const double V = f12 * (a1 / (S + st_i) - a1 / (1.0 + st_i) - a2 / (S + st_j) +
                                a2 / (1.0 + st_j)) +
                         2.0 * (S - d) + a1 / (st_i + S) - a1 / (st_i + d) + a2 / (st_j + S) -
                         a2 / (st_j + d);
        const double Si2 = (S + st_i) * (S + st_i), Sj2 = (S + st_j) * (S + st_j);
        const double dV_dS = f12 * (-a1 / Si2 + a2 / Sj2) + 2.0 - a1 / Si2 - a2 / Sj2;
        const double dV_dd = -2.0 + a1 / ((st_i + d) * (st_i + d)) + a2 / ((st_j + d) * (st_j + d));
        vturb2 = alpha * cs2 * V;
        dvt2_da = cs2 * (V - 0.5 * d * (dV_dd + dV_dS * dS));
    }
    RateDerivs o{0.0, 0.0};
    const double dv2 = r.kbt * (im_i + im_j) + vturb2 + vlam2;
    if (!(dv2 > 0.0)) return o;
    o.Z = (dvt2_da + dvlam2_da) / (2.0 * dv2);
    const double y = 1.5 * r.vf * r.vf / dv2;
    o.X = y < kExpZeroY ? 2.0 * y * y / (1.0 + y) : 0.0;
    return o;
}

// Pair rates of one block of 16 cells (cells cell0 .. cell0 + 15) in the
// 16-cell-blocked layout (blk_elem; cells past C get zeros), double or
// rounded to float, by NT threads of a workgroup: thread t works on cell
// t % 16 and pairs t / 16 + (NT / 16) k, so that the 16 cells of a pair
// leave together (256 contiguous bytes in FP64, 256 bytes in 16-byte steps
// in FP32).  Per-grain values in `lds` as [bin][value][cell]
// (the lanes of a pair read 16 consecutive doubles).  TAB = 7 tabulates St, A,
// B, C and the velocity; for grids whose 16 cells' values would not fit LDS
// otherwise, TAB = 6 leaves out C and TAB = 1 keeps St only (the velocity then
// read from v_dust); what is left out follows from St where it is used, by
// the same arithmetic.  Only pairs in [p0, p1) are written (a block's pairs
// may be shared among several workgroups).
// VI (the vertically integrated kernel) adds one value per grain, h^2, and
// puts the settling speed in the place of the vertical velocity.
template <int TAB, bool VI>
inline size_t rates_blk_lds_bytes(int N) {
    return (size_t)(16 * (TAB + (VI ? 1 : 0)) + 2) * N * sizeof(double);
}

template <int TAB, bool VI, int NT, typename OT>
__device__ void rates_block(const Tables &T, const CellArrays &cells,
                            const double *__restrict__ v_dust, const double *__restrict__ v_frag,
                            OT *__restrict__ K, long C, long cell0, int p0, int p1, double *lds) {
    static_assert(TAB == 7 || TAB == 6 || TAB == 1, "tabulated values per grain");
    static_assert(NT % 64 == 0, "whole waves");
    constexpr int VX = TAB - 3;                       // first velocity row (TAB >= 6)
    constexpr int TW = TAB + (VI ? 1 : 0);            // values per grain; h^2 last
    constexpr int SLOTS = NT / 16;
    const int N = T.N;
    double *tb = lds, *sv = lds + 16 * TW * N, *imv = sv + N;
    // [bin][value][cell]: the values of one grain 128 bytes apart, so that
    // a lane reads them all from one address with immediate offsets
    auto tab = [&](int v, int k, int cl) -> double & { return tb[(k * TW + v) * 16 + cl]; };
    for (int t = threadIdx.x; t < 16 * N; t += NT) {
        const int cl = t & 15, k = t >> 4;
        const long c = cell0 + cl;
        Grain g{};
        if (c < C) {
            const CellRate r = cell_rate(cells, v_frag, c);
            grain_terms(r, T.rho_m, T.s[k], g);
            if (VI) g.h2 = grain_h2(r, g.st);
            if (TAB >= 6) {
                const double *v = v_dust + (c * N + k) * 3;
                g.vx = v[0];
                g.vy = v[1];
                g.vz = VI ? settle_speed(r, g.st, g.h2) : v[2];
            }
        }
        tab(0, k, cl) = g.st;
        if (TAB >= 6) {
            tab(1, k, cl) = g.a;
            tab(2, k, cl) = g.bt;
            if (TAB == 7) tab(3, k, cl) = g.ct;
            tab(VX, k, cl) = g.vx;
            tab(VX + 1, k, cl) = g.vy;
            tab(VX + 2, k, cl) = g.vz;
        }
        if (VI) tab(TAB, k, cl) = g.h2;
    }
    for (int k = threadIdx.x; k < N; k += NT) {
        sv[k] = T.s[k];
        imv[k] = 1.0 / T.m[k];
    }
    __syncthreads();
    const int cl = threadIdx.x & 15, slot = threadIdx.x >> 4;
    const long c = cell0 + cl;
    const bool live = c < C;
    const CellRate r = cell_rate(cells, v_frag, live ? c : C - 1);
    const double *vc = v_dust + (live ? c : C - 1) * N * 3;
    auto grain = [&](int k) {
        Grain g;
        if (TAB >= 6) {
            g.st = tab(0, k, cl);
            g.a = tab(1, k, cl);
            g.bt = tab(2, k, cl);
            if (TAB == 7) g.ct = tab(3, k, cl);
            g.vx = tab(VX, k, cl);
            g.vy = tab(VX + 1, k, cl);
            g.vz = tab(VX + 2, k, cl);
        } else {
            grain_abc(r, tab(0, k, cl), g);
            g.vx = vc[3 * k];
            g.vy = vc[3 * k + 1];
            g.vz = VI ? settle_speed(r, g.st, tab(TAB, k, cl)) : vc[3 * k + 2];
        }
        g.h2 = VI ? tab(TAB, k, cl) : 0.0;
        g.im = imv[k];
        g.s = sv[k];
        return g;
    };
    // the block's base; both kinds of a pair are one 16-byte (FP64) or
    // 8-byte (FP32) store, and a row of odd length gets its zero entry with
    // its diagonal pair
    OT *kb = K + (cell0 / 16) * 64 * pair_slot0(N);
    typedef OT OT2 __attribute__((ext_vector_type(2)));
    uint32_t ijn = p0 + slot < p1 ? T.pij[p0 + slot] : 0u;
    for (int p = p0 + slot; p < p1; p += SLOTS) {
        const uint32_t ij = ijn;
        if (p + SLOTS < p1) ijn = T.pij[p + SLOTS];
        const int i = pair_i(ij), j = pair_j(ij);
        OT oc = (OT)0, of = (OT)0;
        if (live) {
            Grain gi = grain(i);
            const double S = stir_s(r, gi.st);
            if (TAB == 6) gi.ct = gi.st * gi.st / (S + gi.st);
            heavier_terms(r, gi, S);
            double c64, f64;
            pair_rates(r, gi, grain(j), i == j, VI, c64, f64);
            oc = (OT)c64;
            of = (OT)f64;
        }
        const long sl = pair_slot0(i) + (j >> 1);
        *(OT2 *)(kb + blk_elem<OT>(sl, j & 1, cl, 0)) = OT2{oc, of};
        if (i == j && !(i & 1)) *(OT2 *)(kb + blk_elem<OT>(sl, 1, cl, 0)) = OT2{(OT)0, (OT)0};
    }
}

// the table size rates_block takes at N bins (7, 6, or 1 values per grain,
// one more for the vertically integrated kernel)
inline int rates_blk_tab(int N, size_t lds_cap, bool vi) {
    if ((vi ? rates_blk_lds_bytes<7, true>(N) : rates_blk_lds_bytes<7, false>(N)) <= lds_cap)
        return 7;
    if ((vi ? rates_blk_lds_bytes<6, true>(N) : rates_blk_lds_bytes<6, false>(N)) <= lds_cap)
        return 6;
    return 1;
}

}  // namespace coag
