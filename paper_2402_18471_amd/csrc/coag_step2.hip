// coag_step2.hip -- register-resident FP64 right-hand side and step
// (Robinson, Booth & Owen, cuDisc, Sec. 5, eqs. `smol`, `ngain`, `Cijk`,
// `Rijk`, `fragrem`, `Nijk`; BS3(2) sub-cycling of Sec. 5 and Sec. 6).
//
// One workgroup of 8 waves per cell.  The cell's pair rates are read from HBM
// once per coag_step call and stay on chip for every sub-step: Kc in VGPRs,
// Kf in LDS in diagonal-major order (pair (i, j) at D(i - j) + j with
// D(d) = d N - d (d - 1) / 2, so the 64 lanes of a slot read 64 consecutive
// words).
//
// Mapping of the pair triangle: rows in blocks of 64 taken from the top
// (rows [N-64, N), [N-128, N-64), ...); a "slot" is one diagonal d of one row
// block, lane l holding the pair (i, j) = (lo + l, lo + l - d).  The slots of
// all blocks are dealt to the waves in contiguous runs.  Along its run a lane
// keeps the row i fixed and walks j downwards, so
//   * the row-side deposits (coagulation product near bin i, remnant near
//     bin i, loss of grain i, fragments of a destroyed target) stay in
//     registers and are written to LDS only when their target bin changes
//     (the bracketing bin of m_i + m_j only moves down, that of the remnant
//     m_i - chi m_j only up, as j decreases);
//   * the column-side terms (loss of grain j, fragments of a cratering
//     collision, whose top bin depends on j alone) go to lane-distinct LDS
//     addresses, so their atomics never conflict within a wave.
// The two-bin split weights are recomputed from per-bin LDS tables (bin
// masses and 1 / (m_{k+1} - m_k)); no per-pair table is read per evaluation.
#include <hip/hip_runtime.h>
#include <math.h>

#include "coag_device.h"
#include "coag_launch.h"

namespace coag {

constexpr int kWaves2 = 8;
constexpr int kBlock2 = kWaves2 * 64;

__host__ __device__ inline int triangle_slots(int N) {
    int S = 0;
    for (int hi = N; hi > 0; hi -= 64) S += hi;
    return S;
}

// largest k with m[k] <= x (x >= m[0] assumed; returns 0 below)
__device__ __forceinline__ int bin_le(const double *m, int N, double x) {
    int lo = 0, hi = N;                       // m[lo] <= x < m[hi] (m[N] = +inf)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (m[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// LDS view of the per-bin tables of one workgroup
struct BinLds {
    const double *m, *idm, *dE, *invE;
    const int *fcol, *frow, *cdiag, *rdiag;
};

// Per-wave schedule: a run of n slots starting at diagonal d0 of row block b0
// (wave-uniform scalars; later slots follow by stepping d and wrapping into
// the next block).
struct Run {
    int n, b0, d0;
};

__device__ __forceinline__ Run make_run(int N) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int S = triangle_slots(N);
    const int s0 = (int)(((long)w * S) / kWaves2), s1 = (int)(((long)(w + 1) * S) / kWaves2);
    int b = 0, base = 0, hi = N;
    while (s0 >= base + hi) { base += hi; hi -= 64; ++b; }
    return Run{s1 - s0, b, s0 - base};
}

// advance (b, d) to the next slot: rows of block b span diagonals [0, N - 64 b)
__device__ __forceinline__ void next_slot(int N, int &b, int &d) {
    if (++d >= N - 64 * b) { d = 0; ++b; }
}

__device__ __forceinline__ int diag_base(int N, int d) { return d * N - (d * (d - 1)) / 2; }

// Copy one cell's packed-triangle array from HBM into LDS in diagonal-major
// order, kU loads in flight per thread before their stores.
constexpr int kU = 8;
__device__ __forceinline__ void scatter_diag(const Tables &T, const double *__restrict__ src,
                                             double *dst) {
    const int N = T.N, P = T.P;
    for (int base = 0; base < P; base += kU * kBlock2) {
        double v[kU];
        uint32_t ij[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int p = base + u * kBlock2 + threadIdx.x;
            v[u] = p < P ? src[p] : 0.0;
            ij[u] = p < P ? T.pij[p] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int p = base + u * kBlock2 + threadIdx.x;
            const int i = pair_i(ij[u]), j = pair_j(ij[u]);
            if (p < P) dst[diag_base(N, i - j) + j] = v[u];
        }
    }
}

// Rates of the cell on chip.  HBM is read in packed-triangle order (thread t
// takes pairs t, t + 512, ...: fully coalesced) and scattered into LDS in
// diagonal-major order; Kc goes on from LDS into this lane's registers, Kf
// stays in LDS.  Ends with the Kf stores issued (the caller synchronises).
template <int SLOTS>
__device__ __forceinline__ void load_rates(const Tables &T, const Run &r,
                                           const double *__restrict__ Kc,
                                           const double *__restrict__ Kf, double (&kc)[SLOTS],
                                           double *kfl) {
    const int N = T.N, P = T.P;
    const int lane = threadIdx.x & 63;
    scatter_diag(T, Kc, kfl);
    __syncthreads();
    int b = r.b0, d = r.d0;
#pragma clang loop unroll(full)
    for (int t = 0; t < SLOTS; ++t) {
        kc[t] = 0.0;
        if (t < r.n) {
            const int hi = N - 64 * b, lo = hi > 64 ? hi - 64 : 0;
            const int i = lo + lane, j = i - d;
            if (i < hi && j >= 0) kc[t] = kfl[diag_base(N, d) + j];
            next_slot(N, b, d);
        }
    }
    __syncthreads();
    scatter_diag(T, Kf, kfl);
    (void)P;
}

// Per-lane bracket keys of the first pair of this wave's run (row block b0,
// diagonal d0), found once per kernel; later row blocks start at d = 0, whose
// keys come from the per-bin tables cdiag / rdiag.
struct Keys0 {
    int kc, kr;
};

__device__ __forceinline__ Keys0 first_keys(const Tables &T, const BinLds &B, const Run &run) {
    const int N = T.N, lane = threadIdx.x & 63;
    const int hi = N - 64 * run.b0, lo = hi > 64 ? hi - 64 : 0;
    const int i = lo + lane;
    const int ic = i < hi ? i : 0;
    const int j0 = ic - run.d0 >= 0 ? ic - run.d0 : 0;
    const double mi = B.m[ic], mj = B.m[j0];
    const double cm = T.chi * mj;
    // a destroyed target (no remnant) starts from the row's first cratering bracket
    if (!(cm < mi)) return Keys0{bin_le(B.m, N, mi + mj), B.rdiag[ic]};
    const double mr = mi - cm;
    return Keys0{bin_le(B.m, N, mi + mj), mr >= B.m[0] ? bin_le(B.m, N, mr) : 0};
}

// Right-hand side of eq. `smol` for one cell from register-resident rates.
//   y [N] (LDS) in, out [N] (LDS or global) out, w >= 5N + 4 doubles of LDS.
// The slot body is branch-free apart from the rare moves of the two
// bracketing bins; lanes without a pair (masked) deposit exact zeros.
template <int SLOTS, bool NUMBER>
__device__ __forceinline__ void rhs_reg(const Tables &T, const BinLds &B, const Run &run,
                                        const Keys0 &k0, const double (&kc)[SLOTS],
                                        const double *kfl, const double *y, double *out,
                                        double *w) {
    const int N = T.N;
    // keep the per-row set-up below inside the sub-step loop (recomputing it is
    // cheaper than the registers it would hold across the whole loop)
    asm volatile("" ::: "memory");
    double *n = w, *gain = w + N, *phi = w + 2 * N, *loss = w + 3 * N, *suf = w + 4 * N;
    for (int k = threadIdx.x; k < N; k += kBlock2) {
        n[k] = y[k] / B.m[k];
        gain[k] = 0.0;
        phi[k] = 0.0;
        loss[k] = 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const double chi = T.chi;
    const double *m = B.m;

    int cur_b = -1, ic = 0;
    bool rowok = false;
    double ni = 0.0, mi = 0.0;
    double accL = 0.0, aX = 0.0, aY = 0.0, aZ = 0.0, aW = 0.0, aF = 0.0;
    int kcb = 0, krb = 0;                 // current coag / remnant lower bins
    double mcl = 0, mcu = 0, idc = 0;     // m[kcb], m[kcb+1], 1/(m[kcb+1]-m[kcb])
    double mrl = 0, mru = 0, idr = 0;

    auto flush_coag = [&]() {
        atomicAdd(&gain[kcb], aX);
        atomicAdd(&gain[kcb + 1 < N ? kcb + 1 : kcb], aY);
        aX = 0.0;
        aY = 0.0;
    };
    auto flush_rem = [&]() {
        atomicAdd(&gain[krb], aZ);
        atomicAdd(&gain[krb + 1 < N ? krb + 1 : krb], aW);
        aZ = 0.0;
        aW = 0.0;
    };
    // the top bin keeps finite stand-ins for m[k+1] (its weights are selected away)
    auto set_coag = [&](int k) {
        kcb = k;
        mcl = m[k];
        mcu = k + 1 < N ? m[k + 1] : 2.0 * mcl;
        idc = B.idm[k];
    };
    auto set_rem = [&](int k) {
        krb = k;
        mrl = m[k];
        mru = k + 1 < N ? m[k + 1] : 2.0 * mrl;
        idr = B.idm[k];
    };

    struct Ops {
        double nj, mj, kf;
        int fj;
    };
    // operands of a slot that come from LDS, loaded one slot ahead so that
    // their latency overlaps the previous slot's arithmetic and atomics
    auto fetch = [&](int bb, int dd) -> Ops {
        const int hi = N - 64 * bb, lo = hi > 64 ? hi - 64 : 0;
        const int i = lo + lane, j = i - dd;
        const int jc = (i < hi && j >= 0) ? j : 0;
        return Ops{n[jc], m[jc], kfl[diag_base(N, dd) + jc], B.fcol[jc]};
    };
    int b = run.b0, d = run.d0;
    Ops cur = fetch(b, d);
#pragma clang loop unroll(full)
    for (int t = 0; t < SLOTS; ++t) {
        if (t < run.n) {
            if (b != cur_b) {
                if (cur_b >= 0) {
                    flush_coag();
                    flush_rem();
                    atomicAdd(&loss[ic], mi * accL);
                    atomicAdd(&phi[B.frow[ic]], aF);
                    accL = 0.0;
                    aF = 0.0;
                }
                const bool first = cur_b < 0;
                cur_b = b;
                const int hi = N - 64 * b, lo = hi > 64 ? hi - 64 : 0;
                const int i = lo + lane;
                rowok = i < hi;
                ic = rowok ? i : 0;
                ni = n[ic];
                mi = m[ic];
                set_coag(first ? k0.kc : B.cdiag[ic]);
                set_rem(first ? k0.kr : B.rdiag[ic]);
            }
            const int j = ic - d;
            const bool ok = rowok && j >= 0;
            const int jc = ok ? j : 0;
            const double nj = cur.nj, mj = cur.mj, kfv = cur.kf;
            const int fj = cur.fj;
            int b2 = b, d2 = d;
            next_slot(N, b2, d2);
            if (t + 1 < run.n) cur = fetch(b2, d2);
            const double a = ok ? ni * nj : 0.0;
            const double rc = a * kc[t], rf = a * kfv;
            const double sum = rc + rf;
            accL += sum;
            atomicAdd(&loss[jc], mj * sum);
            // coagulation product m_i + m_j between bins kcb, kcb + 1 (all of it
            // in the top bin when it is at or above m_{N-1})
            const double M = mi + mj;
            while (M < mcl && kcb > 0) {
                flush_coag();
                set_coag(kcb - 1);
            }
            {
                const bool top = kcb == N - 1;
                const double eps = (mcu - M) * idc, ome = (M - mcl) * idc;
                const double w0 = top ? M : (NUMBER ? eps * mcl : eps * M);
                const double w1 = top ? 0.0 : (NUMBER ? ome * mcu : ome * M);
                aX += rc * w0;
                aY += rc * w1;
            }
            // cratering remnant m_i - chi m_j between bins krb, krb + 1 (whole at
            // the top bin, or in bin 0 below m_0; zero when the target is destroyed)
            const double cm = chi * mj;
            const bool crater = cm < mi;
            const double Mr = crater ? mi - cm : 0.0;
            while (Mr >= mru && krb < N - 1) {
                flush_rem();
                set_rem(krb + 1);
            }
            {
                const bool whole = krb == N - 1 || Mr < mrl;
                const double eps = (mru - Mr) * idr, ome = (Mr - mrl) * idr;
                const double z0 = whole ? Mr : (NUMBER ? eps * mrl : eps * Mr);
                const double z1 = whole ? 0.0 : (NUMBER ? ome * mru : ome * Mr);
                aZ += rf * z0;
                aW += rf * z1;
            }
            // fragments: total mass minus remnant, collected by the top fragment
            // bin (set by chi m_j when cratering, by m_i when the target is destroyed)
            const double fr = rf * (M - Mr);
            atomicAdd(&phi[fj], crater ? fr : 0.0);
            aF += crater ? 0.0 : fr;
            b = b2;
            d = d2;
        }
    }
    if (cur_b >= 0) {
        flush_coag();
        flush_rem();
        atomicAdd(&loss[ic], mi * accL);
        atomicAdd(&phi[B.frow[ic]], aF);
    }
    __syncthreads();
    // fragments: S_k = sum_{l >= k} phi_l invE_l, each wave scanning 64 bins
    // in parallel, then adding the totals of the chunks above it
    const int wv = threadIdx.x >> 6, nch = (N + 63) >> 6;
    double *tot = suf + N;                          // [nch] chunk totals (in w)
    if (wv < nch) {
        const int k = N - 1 - (64 * wv + lane);    // lane 0: top of the chunk
        double v = k >= 0 ? phi[k] * B.invE[k] : 0.0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double u = __shfl_up(v, o, 64);
            if (lane >= o) v += u;
        }
        if (k >= 0) suf[k] = v;
        if (lane == 63) tot[wv] = v;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += kBlock2) {
        const int ch = (N - 1 - k) >> 6;
        double above = 0.0;
        for (int q = 0; q < ch; ++q) above += tot[q];
        out[k] = (gain[k] + B.dE[k] * (suf[k] + above)) - loss[k];
    }
    __syncthreads();
}

// LDS layout shared by the kernels below
struct Lds2 {
    BinLds B;
    double *kf;        // [P] Kf of the cell, diagonal-major
    double *tail;      // free space after the tables
};

__device__ __forceinline__ Lds2 load_tables(const Tables &T, double *lds) {
    const int N = T.N;
    double *m = lds, *idm = lds + N, *dE = lds + 2 * N, *invE = lds + 3 * N;
    int *fcol = (int *)(lds + 4 * N), *frow = fcol + N, *cdiag = fcol + 2 * N,
        *rdiag = fcol + 3 * N;
    for (int k = threadIdx.x; k < N; k += kBlock2) {
        m[k] = T.m[k];
        idm[k] = T.invdm[k];
        dE[k] = T.dE[k];
        invE[k] = T.invE[k];
        fcol[k] = T.fcol[k];
        frow[k] = T.frow[k];
        cdiag[k] = T.cdiag[k];
        rdiag[k] = T.rdiag[k];
    }
    Lds2 L;
    L.B = BinLds{m, idm, dE, invE, fcol, frow, cdiag, rdiag};
    L.kf = lds + 6 * N;
    L.tail = lds + 6 * N + T.P;
    return L;
}

template <int SLOTS, bool NUMBER>
__global__ __launch_bounds__(kBlock2) void k_rhs2(Tables T, const double *__restrict__ rho,
                                                  const double *__restrict__ Kc,
                                                  const double *__restrict__ Kf,
                                                  double *__restrict__ out) {
    extern __shared__ double lds[];
    const long c = blockIdx.x;
    const int N = T.N;
    const long P = T.P;
    Lds2 L = load_tables(T, lds);
    double *y = L.tail, *f = L.tail + N, *w = L.tail + 2 * N;
    const Run run = make_run(N);
    double kc[SLOTS];
    load_rates<SLOTS>(T, run, Kc + c * P, Kf + c * P, kc, L.kf);
    for (int k = threadIdx.x; k < N; k += kBlock2) y[k] = rho[c * N + k];
    __syncthreads();
    const Keys0 k0 = first_keys(T, L.B, run);
    rhs_reg<SLOTS, NUMBER>(T, L.B, run, k0, kc, L.kf, y, f, w);
    for (int k = threadIdx.x; k < N; k += kBlock2) out[c * N + k] = f[k];
}

// Sub-cycled BS3(2) for one cell per workgroup (same control as k_step).
// The right-hand side is evaluated at a single call site; a stage counter
// says which state it reads and which slope it writes:
//   0: k1 = f(y)           (entry)
//   2: k2 = f(y + h/2 k1)   3: k3 = f(y + 3h/4 k2)
//   4: k4 = f(y+)           (y+ = y + h (2/9 k1 + 1/3 k2 + 4/9 k3))
template <int SLOTS, bool NUMBER>
__global__ __launch_bounds__(kBlock2) void k_step2(Tables T, StepArgs a) {
    extern __shared__ double lds[];
    const long c = blockIdx.x;
    const int N = T.N;
    const long P = T.P;
    Lds2 L = load_tables(T, lds);
    double *y = L.tail, *k1 = y + N, *k2 = y + 2 * N, *k3 = y + 3 * N, *k4 = y + 4 * N,
           *ys = y + 5 * N, *yn = y + 6 * N, *red = y + 7 * N, *w = y + 7 * N + 64;
    const Run run = make_run(N);
    double kc[SLOTS];
    load_rates<SLOTS>(T, run, a.Kc + c * P, a.Kf + c * P, kc, L.kf);
    double *hlog = a.h_log ? a.h_log + c * (long)a.max_sub : nullptr;
    double msum = 0.0;
    for (int k = threadIdx.x; k < N; k += kBlock2) {
        y[k] = a.rho[c * N + k];
        msum += y[k];
    }
    const double mass0 = block_reduce<kBlock2, 0>(msum, red);   // also orders the Kf stores
    const Keys0 k0 = first_keys(T, L.B, run);
    const bool adaptive = a.mode == 0;
    const double dt = a.dt;
    const double atol = a.atol_rel * mass0;
    int nacc = 0, nrej = 0, status = 0;
    int nfix = 0;                                      // FIXED / REPLAY step count
    if (!adaptive) {
        nfix = a.nsub[c];
        if (nfix < 0 || nfix > a.max_sub) { status = 2; nfix = 0; }
    }
    double h = adaptive ? (a.h[c] > 0.0 ? a.h[c] : dt) : 0.0;
    double t = 0.0, hh = 0.0;
    bool clipped = false;

    // set up the next attempt; false when the call is finished
    auto begin = [&]() -> bool {
        if (adaptive) {
            if (!(t < dt)) return false;
            if (nacc + nrej >= a.max_sub) { status = 2; return false; }
            hh = h;
            clipped = false;
            if (hh >= dt - t) { hh = dt - t; clipped = true; }
            if (!clipped && hh < a.h_min_rel * dt) { status = 1; return false; }
        } else {
            if (nacc >= nfix) return false;
            hh = a.mode == 1 ? dt / nfix : hlog[nacc];
        }
        for (int k = threadIdx.x; k < N; k += kBlock2) ys[k] = y[k] + 0.5 * hh * k1[k];
        __syncthreads();
        return true;
    };

    int stage = 0;
    while (true) {
        const double *xin = stage == 0 ? y : stage == 4 ? yn : ys;
        double *kout = stage == 0 ? k1 : stage == 2 ? k2 : stage == 3 ? k3 : k4;
        rhs_reg<SLOTS, NUMBER>(T, L.B, run, k0, kc, L.kf, xin, kout, w);
        if (stage == 0 || stage == 4) {
            if (stage == 4) {
                bool accept = true;
                double fac = 1.0;
                if (adaptive) {
                    double qmax = 0.0, ymin = INFINITY, bad = 0.0;
                    for (int k = threadIdx.x; k < N; k += kBlock2) {
                        const double e = hh * (-5.0 / 72.0 * k1[k] + 1.0 / 12.0 * k2[k] +
                                               1.0 / 9.0 * k3[k] - 1.0 / 8.0 * k4[k]);
                        const double sc = atol + a.rtol * fmax(fabs(y[k]), fabs(yn[k]));
                        if (!isfinite(yn[k]) || !isfinite(e)) bad += 1.0;
                        qmax = fmax(qmax, fabs(e) / sc);
                        ymin = fmin(ymin, yn[k]);
                    }
                    if (block_reduce<kBlock2, 0>(bad, red) > 0.0) { status = 3; break; }
                    const double err = block_reduce<kBlock2, 1>(qmax, red);
                    const double ylo = block_reduce<kBlock2, 2>(ymin, red);
                    if (!isfinite(err)) { status = 3; break; }
                    fac = err == 0.0 ? 5.0 : 0.9 * pow(err, -1.0 / 3.0);
                    fac = fmin(5.0, fmax(0.2, fac));
                    accept = err <= 1.0 && !(ylo < -atol);
                    if (!accept) h = hh * (err <= 1.0 ? 0.5 : fac);
                }
                if (accept) {
                    if (hlog && threadIdx.x == 0 && nacc < a.max_sub && a.mode != 2) hlog[nacc] = hh;
                    ++nacc;
                    if (adaptive) {
                        t = clipped ? dt : t + hh;
                        if (!clipped) h = hh * fac;
                    }
                    for (int k = threadIdx.x; k < N; k += kBlock2) {
                        y[k] = yn[k];
                        k1[k] = k4[k];
                    }
                    __syncthreads();
                } else {
                    ++nrej;
                }
            }
            if (!begin()) break;
            stage = 2;
        } else if (stage == 2) {
            for (int k = threadIdx.x; k < N; k += kBlock2) ys[k] = y[k] + 0.75 * hh * k2[k];
            __syncthreads();
            stage = 3;
        } else {
            for (int k = threadIdx.x; k < N; k += kBlock2)
                yn[k] = y[k] + hh * (2.0 / 9.0 * k1[k] + 1.0 / 3.0 * k2[k] + 4.0 / 9.0 * k3[k]);
            __syncthreads();
            stage = 4;
        }
    }
    if (!adaptive && status == 0) {
        double bad = 0.0;
        for (int k = threadIdx.x; k < N; k += kBlock2) bad += isfinite(y[k]) ? 0.0 : 1.0;
        if (block_reduce<kBlock2, 0>(bad, red) > 0.0) status = 3;
    }
    if (a.renorm && status == 0) {
        double ms = 0.0;
        for (int k = threadIdx.x; k < N; k += kBlock2) ms += y[k];
        const double m1 = block_reduce<kBlock2, 0>(ms, red);
        if (m1 > 0.0) {
            const double sc = mass0 / m1;
            for (int k = threadIdx.x; k < N; k += kBlock2) y[k] *= sc;
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < N; k += kBlock2) a.rho[c * N + k] = y[k];
    if (threadIdx.x == 0) {
        if (adaptive) {
            a.h[c] = h;
            a.nsub[c] = nacc;
        }
        if (a.nrej) a.nrej[c] = nrej;
        a.status[c] = status;
    }
}

// ---------------------------------------------------------------------------
// dispatch on the number of slots each wave holds
// ---------------------------------------------------------------------------
template <typename K>
static hipError_t allow_lds2(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

static size_t rhs2_lds_bytes(int N) {
    return (size_t)(6 * N + N * (N + 1) / 2 + 7 * N + 8) * sizeof(double);
}
static size_t step2_lds_bytes(int N) {
    return (size_t)(6 * N + N * (N + 1) / 2 + 12 * N + 72) * sizeof(double);
}
constexpr size_t kLdsBytes = 160 * 1024;

int reg_slots(int N) {
    const int S = triangle_slots(N);
    return (S + kWaves2 - 1) / kWaves2;
}

#define COAG_SLOT_CASES(X) X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(36) X(40) X(44) X(48)

static int pick_slots(int N) {
    const int need = reg_slots(N);
#define PICK(s) if (need <= s) return s;
    COAG_SLOT_CASES(PICK)
#undef PICK
    return 0;
}

bool reg_path_available(int N) { return pick_slots(N) > 0 && step2_lds_bytes(N) <= kLdsBytes; }

hipError_t launch_rhs2(const Tables &T, long C, const double *rho, const double *Kc,
                       const double *Kf, double *out, hipStream_t st) {
    const size_t bytes = rhs2_lds_bytes(T.N);
    switch (pick_slots(T.N)) {
#define CASE(s)                                                                              \
    case s:                                                                                  \
        if (T.split == 1) {                                                                  \
            if (hipError_t e = allow_lds2(k_rhs2<s, true>, bytes)) return e;                \
            hipLaunchKernelGGL((k_rhs2<s, true>), dim3((unsigned)C), dim3(kBlock2), bytes, st, \
                               T, rho, Kc, Kf, out);                                         \
        } else {                                                                             \
            if (hipError_t e = allow_lds2(k_rhs2<s, false>, bytes)) return e;               \
            hipLaunchKernelGGL((k_rhs2<s, false>), dim3((unsigned)C), dim3(kBlock2), bytes, \
                               st, T, rho, Kc, Kf, out);                                     \
        }                                                                                    \
        break;
        COAG_SLOT_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step2(const Tables &T, long C, const StepArgs &a, hipStream_t st) {
    const size_t bytes = step2_lds_bytes(T.N);
    switch (pick_slots(T.N)) {
#define CASE(s)                                                                              \
    case s:                                                                                  \
        if (T.split == 1) {                                                                  \
            if (hipError_t e = allow_lds2(k_step2<s, true>, bytes)) return e;               \
            hipLaunchKernelGGL((k_step2<s, true>), dim3((unsigned)C), dim3(kBlock2), bytes, \
                               st, T, a);                                                    \
        } else {                                                                             \
            if (hipError_t e = allow_lds2(k_step2<s, false>, bytes)) return e;              \
            hipLaunchKernelGGL((k_step2<s, false>), dim3((unsigned)C), dim3(kBlock2), bytes, \
                               st, T, a);                                                    \
        }                                                                                    \
        break;
        COAG_SLOT_CASES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace coag
