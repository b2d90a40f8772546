// coag_kernels.hip -- FP64 kernels of the gfx950 coagulation-fragmentation
// path (Robinson, Booth & Owen, cuDisc, Sec. 5; sub-cycling of Sec. 6).
//
// Layout: one workgroup per cell; the cell's state, stage vectors and the
// gain / loss / fragment accumulators live in LDS for the whole call, so a
// coag_step launch touches HBM only for the state, the cell's pair rates and
// the redistribution tables (shared by all cells and L2-resident).
#include <hip/hip_runtime.h>
#include <math.h>

#include "coag_device.h"
#include "coag_launch.h"
#include "coag_rate.h"

namespace coag {

// ---------------------------------------------------------------------------
// Redistribution tables (built once per context).  One thread per pair.
// l(M) = largest k with m_k <= M (binary search on the bin masses, so that an
// exact hit goes wholly to its bin); products at or above the top bin go to
// N-1, remnants below bin 0 go to bin 0.
// ---------------------------------------------------------------------------
__device__ int top_fragment_bin(const double *me, int N, double x);

__device__ void split_mass(const double *m, int N, double M, int split, int *k, double *w0,
                           double *w1) {
#pragma clang fp contract(off)
    *k = 0;
    *w0 = 0.0;
    *w1 = 0.0;
    if (!(M > 0.0)) return;
    if (M >= m[N - 1]) { *k = N - 1; *w0 = M; return; }
    if (M < m[0]) { *k = 0; *w0 = M; return; }
    int lo = 0, hi = N - 1;                // m[lo] <= M < m[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (m[mid] <= M) lo = mid; else hi = mid;
    }
    // eps and 1 - eps; the latter as (M - m_l) / (m_u - m_l), free of cancellation
    const double den = m[lo + 1] - m[lo];
    const double eps = (m[lo + 1] - M) / den, ome = (M - m[lo]) / den;
    *k = lo;
    if (split == 1) {                      // NUMBER: one particle split by number
        *w0 = eps * m[lo];
        *w1 = ome * m[lo + 1];
    } else {                               // MASS: mass fractions eps, 1 - eps
        *w0 = eps * M;
        *w1 = ome * M;
    }
}

__global__ void k_build_pairs(int N, const double *__restrict__ m, const double *__restrict__ me,
                              double chi, int split, uint32_t *pij, uint32_t *dst, double *cw0,
                              double *cw1, double *rw0, double *rw1, double *fm) {
#pragma clang fp contract(off)
    const int P = N * (N + 1) / 2;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    // invert p = i(i+1)/2 + j
    int i = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > p) --i;
    while ((i + 1) * (i + 2) / 2 <= p) ++i;
    const int j = p - i * (i + 1) / 2;
    int c, r;
    double a0, a1, b0, b1;
    split_mass(m, N, m[i] + m[j], split, &c, &a0, &a1);
    double mrem, mfmax;
    if (chi * m[j] < m[i]) {               // cratering: remnant of the target
        mrem = m[i] - chi * m[j];
        mfmax = chi * m[j];
    } else {                               // target destroyed
        mrem = 0.0;
        mfmax = m[i];
    }
    split_mass(m, N, mrem, split, &r, &b0, &b1);
    const int f = top_fragment_bin(me, N, mfmax);
    pij[p] = (uint32_t)i | ((uint32_t)j << 10);
    dst[p] = (uint32_t)c | ((uint32_t)r << 10) | ((uint32_t)f << 20);
    cw0[p] = a0;
    cw1[p] = a1;
    rw0[p] = b0;
    rw1[p] = b1;
    fm[p] = (m[i] + m[j]) - mrem;
}

// smallest l with me[l+1] > x, clipped to N-1
__device__ int top_fragment_bin(const double *me, int N, double x) {
    int lo = 0, hi = N;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (me[mid + 1] > x) hi = mid; else lo = mid + 1;
    }
    return lo < N ? lo : N - 1;
}

// Per-bin tables: E_k = (m^e_k)^(2 - eta);  dE_k = E_{k+1} - E_k;
// invE_l = 1 / (E_{l+1} - E_0); 1 / (m_{k+1} - m_k); top fragment bins for a
// largest fragment of chi m_k (cratering) and of m_k (target destroyed).
__global__ void k_build_frag(int N, const double *__restrict__ m, const double *__restrict__ me,
                             double eta, double chi, double *dE, double *invE, double *invdm,
                             int *fcol, int *frow, int *cdiag, int *rdiag) {
#pragma clang fp contract(off)
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const double e0 = pow(me[0], 2.0 - eta);
    const double ek = pow(me[k], 2.0 - eta), ek1 = pow(me[k + 1], 2.0 - eta);
    dE[k] = ek1 - ek;
    invE[k] = 1.0 / (ek1 - e0);
    invdm[k] = k + 1 < N ? 1.0 / (m[k + 1] - m[k]) : 0.0;
    fcol[k] = top_fragment_bin(me, N, chi * m[k]);
    frow[k] = top_fragment_bin(me, N, m[k]);
    // brackets of the diagonal pair (k, k): largest l with m_l <= x
    auto below = [&](double x) {
        int lo = 0, hi = N;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (m[mid] <= x) lo = mid; else hi = mid;
        }
        return lo;
    };
    cdiag[k] = below(m[k] + m[k]);
    // remnant bracket of the first cratering pair of row k (largest j <= k with
    // chi m_j < m_k): the remnant grows as j falls, so every later pair of the
    // row lies at or above it; 0 if the row has none or it is below m_0
    int jr = k;
    while (jr >= 0 && !(chi * m[jr] < m[k])) --jr;
    const double mr = jr >= 0 ? m[k] - chi * m[jr] : 0.0;
    rdiag[k] = mr >= m[0] ? below(mr) : 0;
}

// Pair rates, [C][P], one workgroup of 256 lanes per cell, lane t on pairs
// t, t + 256, ... (a wave writes 64 consecutive pairs), the pair's bins read
// from the pair list one iteration ahead.  The per-grain values of the cell
// sit in LDS.
constexpr int kRatesBlock = 256;

__global__ __launch_bounds__(kRatesBlock) void k_rates(Tables T, CellArrays cells,
                                                       const double *__restrict__ v_dust,
                                                       const double *__restrict__ v_frag,
                                                       double *__restrict__ Kc,
                                                       double *__restrict__ Kf) {
    extern __shared__ double lds[];
    const int N = T.N, P = T.P;
    const long c = blockIdx.x;
    double *St = lds, *A = lds + N, *Bt = lds + 2 * N, *Ct = lds + 3 * N, *Sv = lds + 4 * N,
           *vx = lds + 5 * N, *vy = lds + 6 * N, *vz = lds + 7 * N, *im = lds + 8 * N,
           *sv = lds + 9 * N, *h2 = lds + 10 * N;
    const CellRate r = cell_rate(cells, v_frag, c);
    const bool vert = T.vertical != 0;
    for (int k = threadIdx.x; k < N; k += kRatesBlock) {
        Grain g;
        grain_terms(r, T.rho_m, T.s[k], g);
        St[k] = g.st;
        A[k] = g.a;
        Bt[k] = g.bt;
        Ct[k] = g.ct;
        Sv[k] = stir_s(r, g.st);
        im[k] = 1.0 / T.m[k];
        sv[k] = T.s[k];
        const double *v = v_dust + (c * N + k) * 3;
        vx[k] = v[0];
        vy[k] = v[1];
        if (vert) {
            h2[k] = grain_h2(r, g.st);
            vz[k] = settle_speed(r, g.st, h2[k]);
        } else {
            h2[k] = 0.0;
            vz[k] = v[2];
        }
    }
    __syncthreads();
    auto grain = [&](int k) {
        Grain g;
        g.st = St[k];
        g.a = A[k];
        g.bt = Bt[k];
        g.ct = Ct[k];
        g.vx = vx[k];
        g.vy = vy[k];
        g.vz = vz[k];
        g.im = im[k];
        g.s = sv[k];
        g.h2 = h2[k];
        return g;
    };
    double *kc = Kc + c * P, *kf = Kf + c * P;
    uint32_t ijn = threadIdx.x < P ? T.pij[threadIdx.x] : 0u;
    for (int p = threadIdx.x; p < P; p += kRatesBlock) {
        const uint32_t ij = ijn;
        if (p + kRatesBlock < P) ijn = T.pij[p + kRatesBlock];
        const int i = pair_i(ij), j = pair_j(ij);
        Grain gi = grain(i);
        heavier_terms(r, gi, Sv[i]);
        double c64, f64;
        pair_rates(r, gi, grain(j), i == j, vert, c64, f64);
        kc[p] = c64;
        kf[p] = f64;
    }
}

// Pair rates in the 16-cell-blocked layout, 16 cells per workgroup of 1024
// threads (rates_block); blockIdx.y takes slice y of gridDim.y of the pairs.
template <int TAB, bool VI, typename OT>
__global__ __launch_bounds__(1024) void k_rates_blk(Tables T, CellArrays cells,
                                                    const double *__restrict__ v_dust,
                                                    const double *__restrict__ v_frag,
                                                    OT *__restrict__ K, long C) {
    extern __shared__ double lds[];
    const int P = T.P;
    const int p0 = (int)((long)P * blockIdx.y / gridDim.y);
    const int p1 = (int)((long)P * (blockIdx.y + 1) / gridDim.y);
    rates_block<TAB, VI, 1024>(T, cells, v_dust, v_frag, K, C, (long)blockIdx.x * 16, p0, p1,
                               lds);
}

// ---------------------------------------------------------------------------
// coag_rhs: one workgroup per cell.
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_rhs(Tables T, const double *__restrict__ rho,
                                               const double *__restrict__ Kc,
                                               const double *__restrict__ Kf,
                                               double *__restrict__ out) {
    extern __shared__ double lds[];
    const long c = blockIdx.x;
    const int N = T.N, P = T.P;
    double *y = lds, *f = lds + N, *scratch = lds + 2 * N;
    for (int k = threadIdx.x; k < N; k += BLOCK) y[k] = rho[c * N + k];
    __syncthreads();
    rhs_cell<BLOCK>(T, Kc + c * P, Kf + c * P, y, f, scratch);
    for (int k = threadIdx.x; k < N; k += BLOCK) out[c * N + k] = f[k];
}

// ---------------------------------------------------------------------------
// coag_step: one workgroup per cell, the whole sub-cycle inside the kernel.
// Every thread keeps identical copies of t, h and the counters (they are
// computed from block-wide reductions), so control flow is uniform.
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_step(Tables T, StepArgs a) {
    extern __shared__ double lds[];
    const long c = blockIdx.x;
    const int N = T.N, P = T.P;
    double *y = lds, *k1 = lds + N, *k2 = lds + 2 * N, *k3 = lds + 3 * N, *k4 = lds + 4 * N,
           *ys = lds + 5 * N, *yn = lds + 6 * N, *red = lds + 7 * N,
           *scratch = lds + 7 * N + 64;
    const double *Kc = a.Kc + c * P, *Kf = a.Kf + c * P;
    double *hlog = a.h_log ? a.h_log + c * (long)a.max_sub : nullptr;
    double msum = 0.0;
    for (int k = threadIdx.x; k < N; k += BLOCK) {
        y[k] = a.rho[c * N + k];
        msum += y[k];
    }
    const double mass0 = block_reduce<BLOCK, 0>(msum, red);
    rhs_cell<BLOCK>(T, Kc, Kf, y, k1, scratch);

    int nacc = 0, nrej = 0, status = 0;
    const double dt = a.dt;
    double h = 0.0;

    if (a.mode != 0) {                                   // FIXED or REPLAY
        const int n = a.nsub[c];
        if (n < 0 || n > a.max_sub) {
            status = 2;
        } else {
            for (int sidx = 0; sidx < n; ++sidx) {
                const double hh = a.mode == 1 ? dt / n : hlog[sidx];
                for (int k = threadIdx.x; k < N; k += BLOCK) ys[k] = y[k] + 0.5 * hh * k1[k];
                __syncthreads();
                rhs_cell<BLOCK>(T, Kc, Kf, ys, k2, scratch);
                for (int k = threadIdx.x; k < N; k += BLOCK) ys[k] = y[k] + 0.75 * hh * k2[k];
                __syncthreads();
                rhs_cell<BLOCK>(T, Kc, Kf, ys, k3, scratch);
                for (int k = threadIdx.x; k < N; k += BLOCK)
                    y[k] = y[k] + hh * (2.0 / 9.0 * k1[k] + 1.0 / 3.0 * k2[k] + 4.0 / 9.0 * k3[k]);
                __syncthreads();
                rhs_cell<BLOCK>(T, Kc, Kf, y, k1, scratch);
                if (a.mode == 1 && hlog && threadIdx.x == 0) hlog[sidx] = hh;
            }
            nacc = n;
            double bad = 0.0;
            for (int k = threadIdx.x; k < N; k += BLOCK) bad += isfinite(y[k]) ? 0.0 : 1.0;
            if (block_reduce<BLOCK, 0>(bad, red) > 0.0) status = 3;
        }
    } else {                                             // ADAPTIVE
        const double atol = a.atol_rel * mass0;
        h = a.h[c] > 0.0 ? a.h[c] : dt;
        double t = 0.0;
        while (t < dt) {
            if (nacc + nrej >= a.max_sub) { status = 2; break; }
            double hh = h;
            bool clipped = false;
            if (hh >= dt - t) { hh = dt - t; clipped = true; }
            if (!clipped && hh < a.h_min_rel * dt) { status = 1; break; }
            for (int k = threadIdx.x; k < N; k += BLOCK) ys[k] = y[k] + 0.5 * hh * k1[k];
            __syncthreads();
            rhs_cell<BLOCK>(T, Kc, Kf, ys, k2, scratch);
            for (int k = threadIdx.x; k < N; k += BLOCK) ys[k] = y[k] + 0.75 * hh * k2[k];
            __syncthreads();
            rhs_cell<BLOCK>(T, Kc, Kf, ys, k3, scratch);
            for (int k = threadIdx.x; k < N; k += BLOCK)
                yn[k] = y[k] + hh * (2.0 / 9.0 * k1[k] + 1.0 / 3.0 * k2[k] + 4.0 / 9.0 * k3[k]);
            __syncthreads();
            rhs_cell<BLOCK>(T, Kc, Kf, yn, k4, scratch);
            double qmax = 0.0, ymin = INFINITY, bad = 0.0;
            for (int k = threadIdx.x; k < N; k += BLOCK) {
                const double e = hh * (-5.0 / 72.0 * k1[k] + 1.0 / 12.0 * k2[k] +
                                       1.0 / 9.0 * k3[k] - 1.0 / 8.0 * k4[k]);
                const double sc = atol + a.rtol * fmax(fabs(y[k]), fabs(yn[k]));
                const double q = fabs(e) / sc;
                if (!isfinite(yn[k]) || !isfinite(e)) bad += 1.0;
                qmax = fmax(qmax, q);
                ymin = fmin(ymin, yn[k]);
            }
            if (block_reduce<BLOCK, 0>(bad, red) > 0.0) { status = 3; break; }
            const double err = block_reduce<BLOCK, 1>(qmax, red);
            const double ylo = block_reduce<BLOCK, 2>(ymin, red);
            if (!isfinite(err)) { status = 3; break; }
            double fac = err == 0.0 ? 5.0 : 0.9 * pow(err, -1.0 / 3.0);
            fac = fmin(5.0, fmax(0.2, fac));
            if (err <= 1.0 && !(ylo < -atol)) {
                if (hlog && threadIdx.x == 0 && nacc < a.max_sub) hlog[nacc] = hh;
                ++nacc;
                t = clipped ? dt : t + hh;
                for (int k = threadIdx.x; k < N; k += BLOCK) {
                    y[k] = yn[k];
                    k1[k] = k4[k];
                }
                __syncthreads();
                if (!clipped) h = hh * fac;
            } else {
                ++nrej;
                h = hh * (err <= 1.0 ? 0.5 : fac);
            }
        }
    }
    // optional FP64 mass renormalisation to the entry mass
    if (a.renorm && status == 0) {
        double ms = 0.0;
        for (int k = threadIdx.x; k < N; k += BLOCK) ms += y[k];
        const double m1 = block_reduce<BLOCK, 0>(ms, red);
        if (m1 > 0.0) {
            const double sc = mass0 / m1;
            for (int k = threadIdx.x; k < N; k += BLOCK) y[k] *= sc;
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < N; k += BLOCK) a.rho[c * N + k] = y[k];
    if (threadIdx.x == 0) {
        if (a.mode == 0) {
            a.h[c] = h;
            a.nsub[c] = nacc;
        }
        if (a.nrej) a.nrej[c] = nrej;
        a.status[c] = status;
    }
}

// ---------------------------------------------------------------------------
// Adjoint of a frozen step sequence (one workgroup per cell).
//   Forward replay stores the state at the start of every step in Ys; the
//   reverse sweep recomputes the two intermediate stage states of each step
//   and applies the transposed stage recurrences:
//     mu3 = h 4/9 lam,            v3 = J(y3)^T mu3
//     mu2 = h 1/3 lam + 3h/4 v3,  v2 = J(y2)^T mu2
//     mu1 = h 2/9 lam + h/2 v2,   v1 = J(y)^T mu1,   lam += v1 + v2 + v3.
//   gKc, gKf collect dJ/dKc, dJ/dKf per pair for the rate chain rule.
// ---------------------------------------------------------------------------
// Reverse sweep over the frozen steps of one cell.  The forward replay keeps
// every step's state and its two inner stage states (y2, y3) in the workspace,
// so the sweep evaluates only the three vector-Jacobian products per step.
// dJ/dKc, dJ/dKf are summed over the whole sweep in the global workspace,
// each pair owned by one thread: with only the sweep's 14N doubles in LDS,
// several workgroups share a CU (summing them in LDS instead, 2P more doubles,
// left one workgroup per CU and ran the backward pass 25 % slower).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_adjoint(Tables T, AdjArgs a) {
    extern __shared__ double lds[];
    const long c = blockIdx.x;
    const int N = T.N, P = T.P;
    double *lam = lds, *mu = lds + N, *k1 = lds + 2 * N, *k2 = lds + 3 * N, *k3 = lds + 4 * N,
           *v3 = lds + 6 * N, *v2 = lds + 7 * N, *v1 = lds + 8 * N, *scratch = lds + 9 * N;
    const double *Kc = a.Kc + c * P, *Kf = a.Kf + c * P;
    double *gKc = a.gKc + c * P, *gKf = a.gKf + c * P;
    double *Ys = a.Ys + c * (long)(a.log_stride + 1) * N;
    double *Zs = a.Zs + c * (long)a.log_stride * 2 * N;      // y2, y3 of every step
    const double *hl = a.h_log + c * (long)a.log_stride;
    int n = a.nsub[c];
    const bool ok = n >= 0 && n <= a.log_stride;
    if (!ok) n = 0;
    for (int p = threadIdx.x; p < P; p += BLOCK) {
        gKc[p] = 0.0;
        gKf[p] = 0.0;
    }
    if (!a.replayed)
        for (int k = threadIdx.x; k < N; k += BLOCK) Ys[k] = a.rho_in[c * N + k];
    __syncthreads();
    for (int s = 0; s < (a.replayed ? 0 : n); ++s) {  // forward replay
        const double *y = Ys + (long)s * N;
        double *yn = Ys + (long)(s + 1) * N;
        double *y2 = Zs + (long)s * 2 * N, *y3 = y2 + N;
        const double h = hl[s];
        rhs_cell<BLOCK>(T, Kc, Kf, y, k1, scratch);
        for (int k = threadIdx.x; k < N; k += BLOCK) y2[k] = y[k] + 0.5 * h * k1[k];
        __syncthreads();
        rhs_cell<BLOCK>(T, Kc, Kf, y2, k2, scratch);
        for (int k = threadIdx.x; k < N; k += BLOCK) y3[k] = y[k] + 0.75 * h * k2[k];
        __syncthreads();
        rhs_cell<BLOCK>(T, Kc, Kf, y3, k3, scratch);
        for (int k = threadIdx.x; k < N; k += BLOCK)
            yn[k] = y[k] + h * (2.0 / 9.0 * k1[k] + 1.0 / 3.0 * k2[k] + 4.0 / 9.0 * k3[k]);
        __syncthreads();
    }
    for (int k = threadIdx.x; k < N; k += BLOCK) lam[k] = a.g_out[c * N + k];
    __syncthreads();
    for (int s = n - 1; s >= 0; --s) {
        const double *y = Ys + (long)s * N;
        const double *y2 = Zs + (long)s * 2 * N, *y3 = y2 + N;
        const double h = hl[s];
        for (int k = threadIdx.x; k < N; k += BLOCK) {
            mu[k] = h * (4.0 / 9.0) * lam[k];
            v3[k] = 0.0;
            v2[k] = 0.0;
            v1[k] = 0.0;
        }
        __syncthreads();
        vjp_cell<BLOCK>(T, Kc, Kf, y3, mu, v3, gKc, gKf, scratch);
        for (int k = threadIdx.x; k < N; k += BLOCK) mu[k] = h * (1.0 / 3.0) * lam[k] + 0.75 * h * v3[k];
        __syncthreads();
        vjp_cell<BLOCK>(T, Kc, Kf, y2, mu, v2, gKc, gKf, scratch);
        for (int k = threadIdx.x; k < N; k += BLOCK) mu[k] = h * (2.0 / 9.0) * lam[k] + 0.5 * h * v2[k];
        __syncthreads();
        vjp_cell<BLOCK>(T, Kc, Kf, y, mu, v1, gKc, gKf, scratch);
        for (int k = threadIdx.x; k < N; k += BLOCK) lam[k] += v1[k] + v2[k] + v3[k];
        __syncthreads();
    }
    for (int k = threadIdx.x; k < N; k += BLOCK) a.g_in[c * N + k] = ok ? lam[k] : NAN;
}

// dJ/dalpha and dJ/dv_frag per cell from dJ/dKc, dJ/dKf and the hand-derived
// rate derivatives (clamps of St* and the p_coag branch as in the forward pass).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_rate_grad(Tables T, CellArrays cells,
                                                     const double *__restrict__ v_dust,
                                                     const double *__restrict__ v_frag,
                                                     const double *__restrict__ gKc_all,
                                                     const double *__restrict__ gKf_all,
                                                     double *__restrict__ g_alpha,
                                                     double *__restrict__ g_vfrag) {
    extern __shared__ double lds[];
    const int N = T.N, P = T.P;
    const long c = blockIdx.x;
    double *St = lds, *vx = lds + N, *vy = lds + 2 * N, *vz = lds + 3 * N, *red = lds + 4 * N;
    const double rho_g = cells.rho_g[c], c_s = cells.c_s[c], Om = cells.Omega[c];
    const double v_th = sqrt(8.0 / M_PI) * c_s;
    const double alpha = cells.alpha[c], Tg = cells.T[c], vf = v_frag[c];
    const double delta = 1.0 / sqrt(alpha * c_s * cells.H[c] / cells.nu_mol[c]);
    const double ddelta_da = -0.5 * delta / alpha;
    for (int k = threadIdx.x; k < N; k += BLOCK) {
        St[k] = T.rho_m * T.s[k] / (rho_g * v_th) * Om;
        const double *v = v_dust + (c * N + k) * 3;
        vx[k] = v[0];
        vy[k] = v[1];
        vz[k] = v[2];
    }
    __syncthreads();
    const double *gKc = gKc_all + c * P, *gKf = gKf_all + c * P;
    double ga = 0.0, gv = 0.0;
    for (int p = threadIdx.x; p < P; p += BLOCK) {
        const uint32_t ij = T.pij[p];
        const int i = pair_i(ij), j = pair_j(ij);
        const double St1 = fmax(St[i], St[j]), St2 = fmin(St[i], St[j]);
        double vturb2 = 0.0, dvt2_da = 0.0;
        if (alpha > 0.0) {
            double S = kYStar * St1, dS = 0.0;
            if (S < delta) { S = delta; dS = 1.0; }
            if (S > 1.0) { S = 1.0; dS = 0.0; }
            const double a1 = St1 * St1, a2 = St2 * St2, f12 = (St1 - St2) / (St1 + St2);
            const double dV1 = f12 * (a1 / (S + St1) - a1 / (1.0 + St1) - a2 / (S + St2) + a2 / (1.0 + St2));
            const double dV2 = 2.0 * (S - delta) + a1 / (St1 + S) - a1 / (St1 + delta) +
                               a2 / (St2 + S) - a2 / (St2 + delta);
            const double dV_dS = f12 * (-a1 / ((S + St1) * (S + St1)) + a2 / ((S + St2) * (S + St2))) +
                                 2.0 - a1 / ((St1 + S) * (St1 + S)) - a2 / ((St2 + S) * (St2 + S));
            const double dV_dd = -2.0 + a1 / ((St1 + delta) * (St1 + delta)) +
                                 a2 / ((St2 + delta) * (St2 + delta));
            const double V = dV1 + dV2;
            vturb2 = alpha * c_s * c_s * V;
            dvt2_da = c_s * c_s * V + alpha * c_s * c_s * (dV_dd + dV_dS * dS) * ddelta_da;
        }
        const double mi = T.m[i], mj = T.m[j];
        const double vbm2 = 8.0 * kBoltzmann * Tg * (mi + mj) / (M_PI * mi * mj);
        const double dx = vx[i] - vx[j], dy = vy[i] - vy[j], dz = vz[i] - vz[j];
        const double dv = sqrt(vbm2 + vturb2 + dx * dx + dy * dy + dz * dz);
        const double ddv_da = dvt2_da / (2.0 * dv);
        const double ss = T.s[i] + T.s[j];
        const double sig = M_PI * ss * ss, K = sig * dv;
        const double w = i == j ? 0.5 : 1.0;
        double pf = 0.0, pc = 1.0, dpf_dy = 0.0, y = 0.0;
        if (dv > 0.0) {
            const double q = vf / dv;
            y = 1.5 * q * q;
            const double e = exp(-y);
            pf = (1.0 + y) * e;
            pc = y < kSeriesY ? y * y * (1.0 / 2.0 + y * (-1.0 / 3.0 + y * (1.0 / 8.0 + y * (-1.0 / 30.0 +
                 y * (1.0 / 144.0 + y * (-1.0 / 840.0 + y * (1.0 / 5760.0)))))))
                              : 1.0 - pf;
            dpf_dy = -y * e;
        }
        const double dy_dvf = dv > 0.0 ? 3.0 * vf / (dv * dv) : 0.0;
        const double dy_ddv = dv > 0.0 ? -2.0 * y / dv : 0.0;
        const double dpf_ddv = dpf_dy * dy_ddv;
        const double dKf_da = w * (sig * pf + K * dpf_ddv) * ddv_da;
        const double dKc_da = w * (sig * pc - K * dpf_ddv) * ddv_da;
        const double dKf_dv = w * K * dpf_dy * dy_dvf;
        ga += gKc[p] * dKc_da + gKf[p] * dKf_da;
        gv += (gKf[p] - gKc[p]) * dKf_dv;
    }
    ga = block_reduce<BLOCK, 0>(ga, red);
    gv = block_reduce<BLOCK, 0>(gv, red);
    if (threadIdx.x == 0) {
        g_alpha[c] = ga;
        g_vfrag[c] = gv;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from coag_api.hip).
// ---------------------------------------------------------------------------
constexpr int kBlock = 256;

static size_t lds_bytes(size_t doubles) { return doubles * sizeof(double); }

// Dynamic LDS above 64 KB (large bin counts) has to be requested per kernel.
template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

hipError_t launch_build(int N, const double *m, const double *me, double eta, double chi,
                        int split, uint32_t *pij, uint32_t *dst, double *cw0, double *cw1,
                        double *rw0, double *rw1, double *fm, double *dE, double *invE,
                        double *invdm, int *fcol, int *frow, int *cdiag, int *rdiag,
                        hipStream_t st) {
    const int P = N * (N + 1) / 2;
    hipLaunchKernelGGL(k_build_pairs, dim3((P + 255) / 256), dim3(256), 0, st, N, m, me, chi,
                       split, pij, dst, cw0, cw1, rw0, rw1, fm);
    hipLaunchKernelGGL(k_build_frag, dim3((N + 255) / 256), dim3(256), 0, st, N, m, me, eta, chi,
                       dE, invE, invdm, fcol, frow, cdiag, rdiag);
    return hipGetLastError();
}

hipError_t launch_rates(const Tables &T, long C, const CellArrays &cells, const double *v_dust,
                        const double *v_frag, double *Kc, double *Kf, hipStream_t st) {
    if (C == 0) return hipSuccess;
    const size_t bytes = lds_bytes(11 * T.N);
    if (hipError_t e = allow_lds(k_rates, bytes)) return e;
    hipLaunchKernelGGL(k_rates, dim3((unsigned)C), dim3(kRatesBlock), bytes, st, T, cells, v_dust,
                       v_frag, Kc, Kf);
    return hipGetLastError();
}

template <typename OT>
static hipError_t launch_rates_blk(const Tables &T, long C, const CellArrays &cells,
                                   const double *v_dust, const double *v_frag, OT *K,
                                   hipStream_t st) {
    const unsigned blocks = (unsigned)((C + 15) / 16);
    // few blocks (small grids of cells): share each block's pairs among
    // several workgroups, so that at least ~512 run
    const unsigned slices = blocks >= 512 ? 1u : min(8u, (512u + blocks - 1) / blocks);
    const bool vi = T.vertical != 0;
    const int tab = rates_blk_tab(T.N, 160 * 1024, vi);
#define RATES_BLK(TAB, VI)                                                                        \
    {                                                                                             \
        const size_t bytes = rates_blk_lds_bytes<TAB, VI>(T.N);                                   \
        if (hipError_t e = allow_lds(k_rates_blk<TAB, VI, OT>, bytes)) return e;                  \
        hipLaunchKernelGGL((k_rates_blk<TAB, VI, OT>), dim3(blocks, slices), dim3(1024), bytes,   \
                           st, T, cells, v_dust, v_frag, K, C);                                   \
    }
    if (!vi) {
        if (tab == 7) RATES_BLK(7, false)
        else if (tab == 6) RATES_BLK(6, false)
        else RATES_BLK(1, false)    // fits LDS for every N <= kMaxBins
    } else {
        if (tab == 7) RATES_BLK(7, true)
        else if (tab == 6) RATES_BLK(6, true)
        else RATES_BLK(1, true)
    }
#undef RATES_BLK
    return hipGetLastError();
}

hipError_t launch_rates_blocked(const Tables &T, long C, const CellArrays &cells,
                                const double *v_dust, const double *v_frag, int f32, void *K,
                                hipStream_t st) {
    if (C == 0) return hipSuccess;
    if (f32) return launch_rates_blk(T, C, cells, v_dust, v_frag, (float *)K, st);
    return launch_rates_blk(T, C, cells, v_dust, v_frag, (double *)K, st);
}

hipError_t launch_rhs(const Tables &T, long C, const double *rho, const double *Kc,
                      const double *Kf, double *out, hipStream_t st) {
    if (C == 0) return hipSuccess;
    if (hipError_t e = allow_lds(k_rhs<kBlock>, lds_bytes(7 * T.N))) return e;
    hipLaunchKernelGGL(k_rhs<kBlock>, dim3((unsigned)C), dim3(kBlock), lds_bytes(7 * T.N), st, T,
                       rho, Kc, Kf, out);
    return hipGetLastError();
}

size_t step_lds_bytes(int N) { return lds_bytes(12 * N + 64); }

hipError_t launch_step(const Tables &T, long C, const StepArgs &a, hipStream_t st) {
    if (C == 0) return hipSuccess;
    if (hipError_t e = allow_lds(k_step<kBlock>, step_lds_bytes(T.N))) return e;
    hipLaunchKernelGGL(k_step<kBlock>, dim3((unsigned)C), dim3(kBlock), step_lds_bytes(T.N), st,
                       T, a);
    return hipGetLastError();
}

hipError_t launch_adjoint(const Tables &T, long C, const AdjArgs &a, const CellArrays &cells,
                          const double *v_dust, const double *v_frag, double *g_alpha,
                          double *g_vfrag, hipStream_t st) {
    if (C == 0) return hipSuccess;
    const size_t bytes = lds_bytes(14 * T.N);
    if (hipError_t e = allow_lds(k_adjoint<kBlock>, bytes)) return e;
    hipLaunchKernelGGL(k_adjoint<kBlock>, dim3((unsigned)C), dim3(kBlock), bytes, st, T, a);
    hipLaunchKernelGGL(k_rate_grad<kBlock>, dim3((unsigned)C), dim3(kBlock),
                       lds_bytes(4 * T.N + 64), st, T, cells, v_dust, v_frag, a.gKc, a.gKf,
                       g_alpha, g_vfrag);
    return hipGetLastError();
}

}  // namespace coag
