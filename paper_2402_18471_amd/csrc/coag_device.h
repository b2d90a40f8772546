// coag_device.h -- device-side data structures and per-cell building blocks of
// the gfx950 coagulation-fragmentation path (Robinson, Booth & Owen, cuDisc,
// Sec. 5).  Included by the kernel translation units only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace coag {

constexpr double kBoltzmann = 1.380649e-16;   // erg / K
constexpr double kYStar = 1.6;                // St* / St_1 (intermediate regime)
constexpr double kSeriesY = 1.0e-2;           // p_coag by series below this y
constexpr int kMaxBins = 1023;                // 10-bit bin indices

// Where the products of each packed pair go, built once per context on the
// device (eqs. `Cijk`, `Rijk`, `fragrem`, `Nijk`).  Pair p = i(i+1)/2 + j.
struct Tables {
    int N;
    int P;
    double rho_m;          // grain material density
    const uint32_t *pij;   // [P] i | j << 10
    const uint32_t *dst;   // [P] coag bin | remnant bin << 10 | top fragment bin << 20
    const double *cw0;     // [P] mass to coag bin,        per coagulating collision
    const double *cw1;     // [P] mass to coag bin + 1
    const double *rw0;     // [P] mass to remnant bin,     per fragmenting collision
    const double *rw1;     // [P] mass to remnant bin + 1
    const double *fm;      // [P] fragment mass collected by the top fragment bin
    const double *m;       // [N] bin masses
    const double *s;       // [N] grain radii
    const double *dE;      // [N] E_{k+1} - E_k,   E_k = (m^e_k)^(2 - eta)
    const double *invE;    // [N] 1 / (E_{l+1} - E_0)
    // per-bin tables of the register-resident kernels
    const double *invdm;   // [N] 1 / (m_{k+1} - m_k)  (0 for the top bin)
    const int *fcol;       // [N] top fragment bin when the largest fragment is chi m_j
    const int *frow;       // [N] top fragment bin when the largest fragment is m_i
    const int *cdiag;      // [N] lower bracketing bin of the product m_i + m_i
    const int *rdiag;      // [N] lower bracketing bin of the remnant of the first cratering
                           //     pair (i, j) of row i, the largest such j (0 if none)
    double chi;            // excavated mass / impactor mass
    int split;             // 0 MASS, 1 NUMBER
    int vertical;          // 1: vertically integrated kernel (column densities)
};

// ---------------------------------------------------------------------------
// The 16-cell-blocked rate layout (coag_rates_blocked): per block of 16 cells
// the pairs of each row i are taken two by two, pair (i, j) in slot
// pair_slot0(i) + j / 2 with parity j & 1 (a row of odd length, i even, ends
// with a zero entry (i, i + 1)); pair_slot0(N) slots per block, 64 values per
// slot (2 parities x 16 cells x 2 kinds, Kc then Kf), ordered so that one
// 16-byte load per lane of a wave is contiguous:
//   double: [slot][parity][cell][kind]     float: [slot][cell][parity][kind]
// ---------------------------------------------------------------------------
__host__ __device__ inline long pair_slot0(int i) {
    const long m = i >> 1;
    return (i & 1) ? (m + 1) * (m + 1) : m * (m + 1);
}
template <typename RT>
__host__ __device__ inline long blk_elem(long slot, int parity, int cell, int kind) {
    return sizeof(RT) == 8 ? ((slot * 2 + parity) * 16 + cell) * 2 + kind
                           : ((slot * 16 + cell) * 2 + parity) * 2 + kind;
}

__device__ __forceinline__ int pair_i(uint32_t v) { return v & 1023u; }
__device__ __forceinline__ int pair_j(uint32_t v) { return (v >> 10) & 1023u; }
__device__ __forceinline__ int dst_c(uint32_t v) { return v & 1023u; }
__device__ __forceinline__ int dst_r(uint32_t v) { return (v >> 10) & 1023u; }
__device__ __forceinline__ int dst_f(uint32_t v) { return (v >> 20) & 1023u; }

// ---------------------------------------------------------------------------
// Wavefront / block reductions (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide reduction through `red` (>= BLOCK/64 doubles of LDS).  Every
// thread receives the result.  op: 0 sum, 1 max, 2 min.
template <int BLOCK, int OP>
__device__ __forceinline__ double block_reduce(double v, double *red) {
    constexpr int W = BLOCK / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = OP == 0 ? wave_sum(v) : OP == 1 ? wave_max(v) : wave_min(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int q = 1; q < W; ++q)
        r = OP == 0 ? r + red[q] : OP == 1 ? fmax(r, red[q]) : fmin(r, red[q]);
    return r;
}

// Inclusive suffix sum S_k = sum_{l >= k} x_l over LDS array x[0..N) into
// out[0..N), done by wave 0 in chunks of 64 from the top (carry between
// chunks).  Caller synchronises before and after.
__device__ __forceinline__ void wave0_suffix_sum(const double *x, double *out, int N) {
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    double carry = 0.0;
    for (int top = N - 1; top >= 0; top -= 64) {
        const int k = top - lane;                  // lane 0 holds the highest index
        double v = k >= 0 ? x[k] : 0.0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            double u = __shfl_up(v, o, 64);
            if (lane >= o) v += u;
        }
        v += carry;
        if (k >= 0) out[k] = v;
        carry = __shfl(v, 63, 64);
    }
}

// Inclusive prefix sum P_k = sum_{l <= k} x_l (wave 0, chunks of 64).
__device__ __forceinline__ void wave0_prefix_sum(const double *x, double *out, int N) {
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    double carry = 0.0;
    for (int base = 0; base < N; base += 64) {
        const int k = base + lane;
        double v = k < N ? x[k] : 0.0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            double u = __shfl_up(v, o, 64);
            if (lane >= o) v += u;
        }
        v += carry;
        if (k < N) out[k] = v;
        carry = __shfl(v, 63, 64);
    }
}

// ---------------------------------------------------------------------------
// Right-hand side of eq. `smol` for one cell, one workgroup.
//   y    [N] state (LDS or global), out [N] result (LDS or global)
//   lds  >= 5N doubles of LDS scratch: n, gain, phi, loss, suffix
// Gain and loss are scattered with LDS FP64 atomics; fragments are collected
// per top bin and then distributed with the power-law fractions through one
// suffix sum:  G_k += dE_k sum_{l >= k} phi_l invE_l.
// ---------------------------------------------------------------------------
template <int BLOCK>
__device__ void rhs_cell(const Tables &T, const double *__restrict__ Kc,
                         const double *__restrict__ Kf, const double *y, double *out,
                         double *lds) {
    const int N = T.N, P = T.P;
    double *n = lds, *gain = lds + N, *phi = lds + 2 * N, *loss = lds + 3 * N,
           *suf = lds + 4 * N;
    for (int k = threadIdx.x; k < N; k += BLOCK) {
        n[k] = y[k] / T.m[k];
        gain[k] = 0.0;
        phi[k] = 0.0;
        loss[k] = 0.0;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += BLOCK) {
        const uint32_t ij = T.pij[p], d = T.dst[p];
        const int i = pair_i(ij), j = pair_j(ij);
        const double a = n[i] * n[j];
        const double kc = Kc[p], kf = Kf[p];
        const double rc = a * kc, rf = a * kf;
        const int c = dst_c(d), r = dst_r(d), f = dst_f(d);
        atomicAdd(&gain[c], rc * T.cw0[p]);
        const double cw1 = T.cw1[p];
        if (cw1 != 0.0) atomicAdd(&gain[c + 1], rc * cw1);
        const double rw0 = T.rw0[p], rw1 = T.rw1[p];
        if (rw0 != 0.0) atomicAdd(&gain[r], rf * rw0);
        if (rw1 != 0.0) atomicAdd(&gain[r + 1], rf * rw1);
        atomicAdd(&phi[f], rf * T.fm[p]);
        // loss of both partners with the un-halved kernel (Kc, Kf carry w = 1/2
        // on the diagonal, where the pair is counted once)
        const double kt = (i == j) ? 2.0 * (rc + rf) : (rc + rf);
        atomicAdd(&loss[i], T.m[i] * kt);
        if (i != j) atomicAdd(&loss[j], T.m[j] * kt);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += BLOCK) phi[k] *= T.invE[k];
    __syncthreads();
    wave0_suffix_sum(phi, suf, N);
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += BLOCK)
        out[k] = (gain[k] + T.dE[k] * suf[k]) - loss[k];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Vector-Jacobian product of the right-hand side for one cell:
//   gy[k]  += sum (d f / d y_k) mu          (LDS, accumulated)
//   gKc[p] += a_p (mu . (Dc_p - l_p)),  gKf[p] += a_p (mu . (Df_p - l_p))
// where f = sum_p a_p (Kc_p (Dc_p - l_p) + Kf_p (Df_p - l_p)), a_p = n_i n_j,
// D the redistribution rows and l_p the partners' loss masses / w_p.
// Each pair is owned by one thread (gKc/gKf need no atomics).
//   lds >= 4N doubles: n, gn, t1, t2
// ---------------------------------------------------------------------------
template <int BLOCK>
__device__ void vjp_cell(const Tables &T, const double *__restrict__ Kc,
                         const double *__restrict__ Kf, const double *y, const double *mu,
                         double *gy, double *__restrict__ gKc, double *__restrict__ gKf,
                         double *lds) {
    const int N = T.N, P = T.P;
    double *n = lds, *gn = lds + N, *t1 = lds + 2 * N, *pre = lds + 3 * N;
    for (int k = threadIdx.x; k < N; k += BLOCK) {
        n[k] = y[k] / T.m[k];
        gn[k] = 0.0;
        t1[k] = mu[k] * T.dE[k];
    }
    __syncthreads();
    wave0_prefix_sum(t1, pre, N);      // pre_l = sum_{k<=l} mu_k dE_k
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += BLOCK) {
        const uint32_t ij = T.pij[p], d = T.dst[p];
        const int i = pair_i(ij), j = pair_j(ij);
        const int c = dst_c(d), r = dst_r(d), f = dst_f(d);
        const double cw1 = T.cw1[p], rw0 = T.rw0[p], rw1 = T.rw1[p];
        double dc = mu[c] * T.cw0[p];
        if (cw1 != 0.0) dc += mu[c + 1] * cw1;
        double df = T.fm[p] * pre[f] * T.invE[f];
        if (rw0 != 0.0) df += mu[r] * rw0;
        if (rw1 != 0.0) df += mu[r + 1] * rw1;
        const double lp = (i == j) ? 2.0 * mu[i] * T.m[i] : mu[i] * T.m[i] + mu[j] * T.m[j];
        const double sc = dc - lp, sf = df - lp;
        const double a = n[i] * n[j];
        gKc[p] += a * sc;
        gKf[p] += a * sf;
        const double ga = Kc[p] * sc + Kf[p] * sf;
        atomicAdd(&gn[i], n[j] * ga);
        atomicAdd(&gn[j], n[i] * ga);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += BLOCK) gy[k] += gn[k] / T.m[k];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Pair rates (eqs. `kernel`, `vbrown`, `OCVrel`, `p_frag`).
// Per-cell quantities are passed in; St_i, St_j are the pair's Stokes numbers.
// ---------------------------------------------------------------------------
struct CellState {
    double T, c_s, alpha, delta, v_frag;
};

struct PairRate {
    double Kc, Kf;
};

__device__ __forceinline__ PairRate pair_rate(const CellState &cs, double St_i, double St_j,
                                              double m_i, double m_j, double s_i, double s_j,
                                              double vlam2, double w) {
    const double St1 = St_i >= St_j ? St_i : St_j;
    const double St2 = St_i >= St_j ? St_j : St_i;
    double vturb2 = 0.0;
    if (cs.alpha > 0.0) {
        const double delta = cs.delta;
        double S = kYStar * St1;
        if (S < delta) S = delta;
        if (S > 1.0) S = 1.0;
        const double a1 = St1 * St1, a2 = St2 * St2;
        const double dV1 = (St1 - St2) / (St1 + St2) *
                           (a1 / (S + St1) - a1 / (1.0 + St1) - a2 / (S + St2) + a2 / (1.0 + St2));
        const double dV2 = 2.0 * (S - delta) + a1 / (St1 + S) - a1 / (St1 + delta) +
                           a2 / (St2 + S) - a2 / (St2 + delta);
        vturb2 = cs.alpha * cs.c_s * cs.c_s * (dV1 + dV2);
    }
    const double vbm2 = 8.0 * kBoltzmann * cs.T * (m_i + m_j) / (M_PI * m_i * m_j);
    const double dv = sqrt(vbm2 + vturb2 + vlam2);
    const double ss = s_i + s_j;
    const double K = M_PI * ss * ss * dv;
    double pf, pc;
    if (dv == 0.0) {
        pf = 0.0;
        pc = 1.0;
    } else {
        const double q = cs.v_frag / dv;
        const double y = 1.5 * q * q;
        pf = (1.0 + y) * exp(-y);
        if (y < kSeriesY) {
            pc = y * y * (1.0 / 2.0 + y * (-1.0 / 3.0 + y * (1.0 / 8.0 + y * (-1.0 / 30.0 +
                 y * (1.0 / 144.0 + y * (-1.0 / 840.0 + y * (1.0 / 5760.0)))))));
        } else {
            pc = 1.0 - pf;
        }
    }
    return PairRate{w * K * pc, w * K * pf};
}

}  // namespace coag
