// coag_adjoint.hip -- the cell-batched discrete adjoint of coag_step over a
// frozen step sequence, with the transposed gain contraction on the matrix
// cores.
//
// The right-hand side of eq. `smol` for one cell is bilinear in the number
// densities and the pair rates: with a_p = n_i n_j for pair p = (i, j),
//   f = sum_p a_p (Kc_p (Dc_p - l_p) + Kf_p (Df_p - l_p)),
// Dc_p, Df_p the redistribution rows (eqs. `Cijk`, `Rijk`, `fragrem`, `Nijk`)
// and l_p the loss of both partners (m_i, m_j at bins i, j).  For a cotangent
// mu of f its transpose gives, per pair,
//   sc_p = mu . (Dc_p - l_p),   sf_p = mu . (Df_p - l_p),
//   ga_p = Kc_p sc_p + Kf_p sf_p,
//   dJ/dn_i += n_j ga_p,  dJ/dn_j += n_i ga_p,
//   dJ/dKc_p += a_p sc_p,  dJ/dKf_p += a_p sf_p.
// A workgroup of 8 waves takes 16 cells.  The part of mu . D_p inside the
// 16-bin window of row i (coagulation and remnant products, and the heavier
// grain's loss m_i, folded into D as in the forward step) is a matrix product
// S[pair, cell] = sum_bin D[pair, bin] mu[cell, bin] per chunk of 16 pairs of
// one row: FP64 matrix cores, or split BF16 (three limbs of D and of mu
// scaled by a power of two per cell, six limb products in FP32, read back in
// FP64 per chunk).  The lighter grain's loss mu_j m_j and the fragments (mass
// of the pair's fragments times invE_l sum_{k <= l} mu_k dE_k at the top
// fragment bin l, the transpose of the per-top-bin accumulation) are FP64
// vector terms.  dJ/dKc, dJ/dKf are never stored: each pair's terms are
// folded at once into the cell's dJ/dalpha and dJ/dv_frag through the rate
// derivatives, which follow from the rates and two per-pair factors Z, X
// (pair_rate_derivs) that a pre-pass writes per call next to the rates:
//   dJ/dalpha  += Z (a ga + D),   dJ/dv_frag += -D / v_frag,
//   D = a X Kf (sf - sc);
// the vertically integrated kernel adds W a ga to dJ/dalpha, W = d ln G /
// d alpha of its overlap factor G (a third per-pair factor).
//
// The reverse sweep of one BS3 step of size h from the adjoint state lambda
// (the transposed stage recurrences):
//   mu3 = 4h/9 lambda,               v3 = J(y3)^T mu3
//   mu2 = h/3 lambda + 3h/4 v3,      v2 = J(y2)^T mu2
//   mu1 = 2h/9 lambda + h/2 v2,      v1 = J(y)^T mu1
//   lambda <- lambda + (v3 + v2) + v1.
// The step-start states y and stage states y2, y3 come from the forward
// replay (the batched step in REPLAY mode).  The 16 cells sweep in lockstep,
// aligned at their last step; a cell whose steps are done takes mu = 0,
// n = 0, which contributes nothing.
#include <hip/hip_runtime.h>
#include <math.h>

#include "coag_batch.h"
#include "coag_batch_common.h"
#include "coag_rate.h"

namespace coag {

namespace {

using namespace bc;

// ---------------------------------------------------------------------------
// Rate-derivative factors Z, X (and W for the vertically integrated kernel,
// VI) in the 16-cell-blocked layout: 16 cells per workgroup of 1024 threads,
// thread t on cell t % 16 and pairs t / 16 + 64 k (the 16 cells of a pair
// leave as one run).  Per-grain St and velocity of the 16 cells in LDS as
// [bin][value][cell] (TAB = 4), or St alone (TAB = 1, velocities from v_dust)
// where that would not fit; VI adds h^2 and e = d ln h / d alpha per grain,
// and its vertical velocity is the settling speed.
// ---------------------------------------------------------------------------
template <int TAB, bool VI>
size_t derivs_lds_bytes(int N) {
    return (size_t)(16 * (TAB + (VI ? 2 : 0)) + 1) * N * sizeof(double);
}

template <int TAB, bool VI, typename GT>
__global__ __launch_bounds__(1024) void k_rate_derivs_blk(Tables T, CellArrays cells,
                                                          const double *__restrict__ v_dust,
                                                          const double *__restrict__ v_frag,
                                                          GT *__restrict__ Zo,
                                                          GT *__restrict__ Xo,
                                                          GT *__restrict__ Wo, long C) {
    extern __shared__ double lds[];
    constexpr int TW = TAB + (VI ? 2 : 0);             // values per grain; h^2, e last
    const int N = T.N, P = T.P;
    const long cell0 = (long)blockIdx.x * 16;
    double *tb = lds, *imv = lds + 16 * TW * N;
    auto tab = [&](int v, int k, int cl) -> double & { return tb[(k * TW + v) * 16 + cl]; };
    for (int t = threadIdx.x; t < 16 * N; t += 1024) {
        const int cl = t & 15, k = t >> 4;
        const long c = cell0 + cl;
        double st = 0.0, vx = 0.0, vy = 0.0, vz = 0.0, h2 = 0.0, e = 0.0;
        if (c < C) {
            const CellRate r = cell_rate(cells, v_frag, c);
            st = T.rho_m * T.s[k] / r.rg_vth * r.Om;
            if (VI) {
                h2 = grain_h2(r, st);
                e = vertical_e(r, st);
            }
            if (TAB == 4) {
                const double *v = v_dust + (c * N + k) * 3;
                vx = v[0];
                vy = v[1];
                vz = VI ? settle_speed(r, st, h2) : v[2];
            }
        }
        tab(0, k, cl) = st;
        if (TAB == 4) {
            tab(1, k, cl) = vx;
            tab(2, k, cl) = vy;
            tab(3, k, cl) = vz;
        }
        if (VI) {
            tab(TAB, k, cl) = h2;
            tab(TAB + 1, k, cl) = e;
        }
    }
    for (int k = threadIdx.x; k < N; k += 1024) imv[k] = 1.0 / T.m[k];
    __syncthreads();
    const int p0 = (int)((long)P * blockIdx.y / gridDim.y);
    const int p1 = (int)((long)P * (blockIdx.y + 1) / gridDim.y);
    const int cl = threadIdx.x & 15, slot = threadIdx.x >> 4;
    const long c = cell0 + cl;
    const bool live = c < C;
    const long cc = live ? c : C - 1;
    const CellRate r = cell_rate(cells, v_frag, cc);
    const double alpha = cells.alpha[cc], cs = cells.c_s[cc], cs2 = cs * cs;
    const double *vc = v_dust + cc * N * 3;
    auto vel = [&](int k, int d) {
        if (TAB == 4) return tab(1 + d, k, cl);
        if (VI && d == 2) return settle_speed(r, tab(0, k, cl), tab(TAB, k, cl));
        return vc[3 * k + d];
    };
    GT *oz = Zo + cell0 * P + cl, *ox = Xo + cell0 * P + cl;
    for (int p = p0 + slot; p < p1; p += 64) {
        RateDerivs d{0.0, 0.0};
        double w = 0.0;
        if (live) {
            const uint32_t ij = T.pij[p];
            const int i = pair_i(ij), j = pair_j(ij);
            const double vzi = vel(i, 2), vzj = vel(j, 2);
            const double dx = vel(i, 0) - vel(j, 0), dy = vel(i, 1) - vel(j, 1), dz = vzi - vzj;
            double dvlam2_da = 0.0;
            if (VI) {
                const double ei = tab(TAB + 1, i, cl), ej = tab(TAB + 1, j, cl);
                dvlam2_da = 2.0 * dz * (vzi * ei - vzj * ej);
                w = vertical_w(tab(TAB, i, cl), ei, tab(TAB, j, cl), ej);
            }
            d = pair_rate_derivs(r, alpha, cs2, tab(0, i, cl), tab(0, j, cl), imv[i], imv[j],
                                 dx * dx + dy * dy + dz * dz, dvlam2_da);
        }
        oz[(long)p * 16] = (GT)d.Z;
        ox[(long)p * 16] = (GT)d.X;
        if (VI) Wo[cell0 * P + cl + (long)p * 16] = (GT)w;
    }
}

// ---------------------------------------------------------------------------
// The reverse sweep, 16 cells per workgroup.
// ---------------------------------------------------------------------------
struct ACtl {
    double mus;          // split form: FP64 value of one unit of the cell's scaled FP32 mu
    int n, bad;          // steps of the cell; its inputs are invalid (outputs NaN)
};

// LDS: nv (n of the stage state), mu, qf (fragment cotangent per top bin) and
// gn (dJ/dn accumulated by the contraction), each [16][NS] FP64; per bin m and
// three int tables; the split form's scaled FP32 mu [16][NS]; control words.
struct AdjLds {
    size_t nv, mu, qf, gn, mk, fcol, frow, wbl, muf, ctl, red, nmax, total;
};

__host__ __device__ inline AdjLds adj_lds_layout(int N, int prec) {
    const size_t NS = (size_t)batch_row_stride(N);
    AdjLds L;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += (b + 15) & ~size_t(15); return r; };
    L.nv = take(kBC * NS * 8);
    L.mu = take(kBC * NS * 8);
    L.qf = take(kBC * NS * 8);
    L.gn = take(kBC * NS * 8);
    L.mk = take((size_t)N * 8);
    L.fcol = take((size_t)N * 4);
    L.frow = take((size_t)N * 4);
    L.wbl = take((size_t)N * 4);
    L.muf = take(prec == 1 ? kBC * NS * 4 : 0);
    L.ctl = take(kBC * sizeof(ACtl));
    L.red = take(2 * kBC * 8);
    L.nmax = take(16);
    L.total = o;
    return L;
}

constexpr int kRingA = 2;
static_assert(kRingA % 2 == 0, "the D operands alternate between two register sets by chunk parity");

template <int PREC, typename RT, typename GT, bool VI>
__global__ __launch_bounds__(kBBlock) void k_adj_batch(Tables T, BatchTables B, AdjBatchArgs a,
                                                       long C) {
    extern __shared__ double lds_d[];
    char *lds = (char *)lds_d;
    const int N = T.N;
    const long P = T.P;
    const long bt = batch_of(blockIdx.x, gridDim.x);
    const long cell0 = bt * kBC;
    const int NS = batch_row_stride(N);
    const AdjLds LL = adj_lds_layout(N, PREC);
    double *nv = (double *)(lds + LL.nv), *mu = (double *)(lds + LL.mu),
           *qf = (double *)(lds + LL.qf), *gn = (double *)(lds + LL.gn),
           *mk = (double *)(lds + LL.mk);
    int *fcol = (int *)(lds + LL.fcol), *frow = (int *)(lds + LL.frow),
        *wbl = (int *)(lds + LL.wbl);
    float *muf = (float *)(lds + LL.muf);
    ACtl *ctl = (ACtl *)(lds + LL.ctl);
    double *red = (double *)(lds + LL.red);
    int *nmaxp = (int *)(lds + LL.nmax);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int L = a.L;

    for (int k = threadIdx.x; k < N; k += kBBlock) {
        mk[k] = T.m[k];
        fcol[k] = T.fcol[k];
        frow[k] = T.frow[k];
        wbl[k] = B.wb[k];
    }
    for (int t = threadIdx.x; t < kBC * NS; t += kBBlock) gn[t] = 0.0;
    if (threadIdx.x == 0) *nmaxp = 0;
    if (threadIdx.x < 2 * kBC) red[threadIdx.x] = 0.0;
    __syncthreads();
    // ---- set-up: each wave owns cells wv and wv + 8; lambda lives in g_in ----
    for (int u = 0; u < 2; ++u) {
        const int c = wv + 8 * u;
        const long gc = cell0 + c;
        const bool live = gc < C;
        int n = live ? a.nsub[gc] : 0;
        const bool bad = live && (n < 0 || n > L || a.status[gc] != 0);
        if (bad) n = 0;
        if (live)
            for (int k = lane; k < N; k += 64) a.g_in[gc * N + k] = a.g_out[gc * N + k];
        if (lane == 0) {
            ctl[c].n = n;
            ctl[c].bad = bad;
            ctl[c].mus = 0.0;
            atomicMax(nmaxp, n);
        }
    }
    __syncthreads();
    const int maxn = *nmaxp;

    // ---- stage algebra of cell c before contraction v (3, 2, 1) of sweep
    // iteration t (owner wave); v = 0 with t = maxn: the last update ----
    auto prepare = [&](int c, int t, int v) {
        const long gc = cell0 + c;
        if (gc >= C) {
            for (int k = lane; k < N; k += 64) {
                nv[c * NS + k] = 0.0;
                mu[c * NS + k] = 0.0;
                qf[c * NS + k] = 0.0;
                gn[c * NS + k] = 0.0;
                if (PREC == 1) muf[c * NS + k] = 0.0f;
            }
            return;
        }
        const int n = ctl[c].n;
        const bool act = v > 0 && t < n;                  // this stage's step exists
        const bool prev = v == 3 || v == 0 ? t >= 1 && t - 1 < n : false;  // v1 pending
        const int s = n - 1 - t;
        const double h = act ? a.h_log[gc * L + s] : 0.0;
        const double *y = nullptr;
        if (act)
            y = v == 1 ? a.Ys + (gc * (L + 1) + s) * (long)N
                       : a.Zs + ((gc * L + s) * 2 + (v == 3 ? 1 : 0)) * (long)N;
        double *lam = a.g_in + gc * N, *v3w = a.v3 + gc * N;
        double mx = 0.0;
        for (int k = lane; k < N; k += 64) {
            const double gv = gn[c * NS + k] / mk[k];       // v of the last contraction
            double muk = 0.0, nk = 0.0;
            if (v == 3 || v == 0) {
                double l = lam[k];
                if (prev) {
                    l += gv;                                 // lambda += v1
                    lam[k] = l;
                }
                if (act) muk = h * (4.0 / 9.0) * l;
            } else if (v == 2) {
                if (act) {
                    v3w[k] = gv;
                    muk = h * (1.0 / 3.0) * lam[k] + 0.75 * h * gv;
                }
            } else if (act) {
                const double l = lam[k];
                muk = h * (2.0 / 9.0) * l + 0.5 * h * gv;
                lam[k] = l + (v3w[k] + gv);                  // lambda += v3 + v2
            }
            if (act) nk = y[k] / mk[k];
            nv[c * NS + k] = nk;
            mu[c * NS + k] = muk;
            gn[c * NS + k] = 0.0;
            mx = fmax(mx, fabs(muk));
        }
        // fragment cotangent per top bin l: invE_l sum_{k <= l} mu_k dE_k
        double carry = 0.0;
        for (int base = 0; base < N; base += 64) {
            const int k = base + lane;
            double x = k < N ? mu[c * NS + k] * T.dE[k] : 0.0;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const double yv = __shfl_up(x, o, 64);
                if (lane >= o) x += yv;
            }
            if (k < N) qf[c * NS + k] = (x + carry) * T.invE[k];
            carry += __shfl(x, 63, 64);
        }
        if (PREC == 1) {
            // scale by a power of two so that |mu| <= 1 in FP32
            mx = wave_max_d(mx);
            const int e = mx > 0.0 ? ilogb(mx) + 1 : 0;
            const double sc = mx > 0.0 ? ldexp(1.0, -e) : 0.0;
            for (int k = lane; k < N; k += 64) muf[c * NS + k] = (float)(mu[c * NS + k] * sc);
            if (lane == 0) ctl[c].mus = mx > 0.0 ? ldexp(1.0, e) : 0.0;
        }
    };

    // ---- one transposed right-hand side of all 16 cells.  Chunks in
    // column-block order (q outer, row i inner), each wave a contiguous range,
    // so a lane keeps its lighter grains j over many chunks: their loss
    // cotangents mu_j m_j, crater fragment cotangents and their dJ/dn_j sums
    // sit in registers and the sums are deposited when the block changes;
    // the heavier grain's dJ/dn_i takes one LDS atomic per lane and chunk.
    // Rates and derivatives are loaded kRingA chunks ahead into a register
    // ring, D operands one chunk ahead, every load unconditional. ----
    // this lane's share of dJ/dalpha and of -v_frag dJ/dv_frag of cell cl
    double gacc_a = 0.0, gacc_v = 0.0;
    auto contract = [&]() {
        const int cl = lane & 15, g = lane >> 4;
        const int NC = B.NC;
        const int c0 = (int)((long)wv * NC / kBWaves), c1 = (int)((long)(wv + 1) * NC / kBWaves);
        if (c0 >= c1) return;
        const double chi = T.chi;
        const double *nrow = nv + cl * NS, *murow = mu + cl * NS, *qrow = qf + cl * NS;
        double *gnrow = gn + cl * NS;
        const double mus = PREC == 1 ? ctl[cl].mus : 1.0;
        // the pair of MFMA output register r: row g + 4r (FP64 16x16x4),
        // 4g + r (BF16 16x16x32)
        auto pj = [&](int r) { return PREC == 0 ? g + 4 * r : 4 * g + r; };
        auto advance = [N](int &i, int &q) {
            if (i + 1 < N) ++i;
            else { ++q; i = 16 * q; }
        };
        const int cr0 = __builtin_amdgcn_readfirstlane(B.crow_c[c0]);
        int ci = cr0 & 0xffff, cq = cr0 >> 16;
        int ri = ci, rq = cq;
        // lighter grains of the lane in the current column block
        double njr[4], mjr[4], lmu[4], qcr[4], col[4];
        int colq = cq;
        auto load_block = [&](int q) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 16 * q + pj(r);
                const bool in = j < N;
                const int jj = in ? j : N - 1;
                njr[r] = in ? nrow[jj] : 0.0;
                mjr[r] = mk[jj];
                lmu[r] = in ? murow[jj] * mjr[r] : 0.0;
                qcr[r] = qrow[fcol[jj]];
                col[r] = 0.0;
            }
        };
        auto flush_block = [&](int q) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 16 * q + pj(r);
                if (j < N) atomicAdd(&gnrow[j], col[r]);
            }
        };
        load_block(colq);
        // the batch's arrays from uniform bases with 32-bit lane offsets: the
        // rates in the blocked layout of coag_rates_blocked (blk_elem; one
        // 16-byte load per pair in FP64, per two pairs in FP32), the
        // derivative factors [P][16] (pair p of cell cl at p * 16 + cl)
        const long kbase = cell0 * P;
        const RT *Kb = (const RT *)a.Kc + cell0 / kBC * 64 * pair_slot0(N);
        const __amdgpu_buffer_rsrc_t kr =
            raw_buffer(Kb, (unsigned)(64 * pair_slot0(N) * sizeof(RT)));
        const GT *Zp = (const GT *)a.Z + kbase, *Xp = (const GT *)a.X + kbase;
        const GT *Wp = VI ? (const GT *)a.W + kbase : nullptr;
        RT rc[kRingA][4], rf[kRingA][4];
        GT ez[kRingA][4], ex[kRingA][4], ew[kRingA][VI ? 4 : 1];
        auto load_k = [&](int i, int q, int u) {
            const int prow = i * (i + 1) / 2;
            const unsigned s0 = (unsigned)pair_slot0(i);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 16 * q + pj(r), jc = j <= i ? j : i;
                const unsigned o = (unsigned)(prow + jc) * 16u + (unsigned)cl;
                if constexpr (sizeof(RT) == 8) {
                    const unsigned ob =
                        (unsigned)blk_elem<double>(s0 + (jc >> 1), jc & 1, cl, 0) * 8u;
                    const f64x2 v = buf_f64x2<false>(kr, ob);
                    rc[u][r] = v[0];
                    rf[u][r] = v[1];
                } else if ((r & 1) == 0) {
                    // pairs 4g + r, 4g + r + 1 (r even) from one slot; pairs
                    // past the diagonal are masked where they are used
                    const unsigned ob =
                        (unsigned)blk_elem<float>(s0 + (jc >> 1), 0, cl, 0) * 4u;
                    const f32x4 v = buf_f32x4<false>(kr, ob);
                    rc[u][r] = v[0];
                    rf[u][r] = v[1];
                    rc[u][r + 1] = v[2];
                    rf[u][r + 1] = v[3];
                }
                ez[u][r] = Zp[o];
                ex[u][r] = Xp[o];
                if (VI) ew[u][VI ? r : 0] = Wp[o];
            }
        };
        int rleft = c1 - c0;
        auto next_k = [&](int u) {
            load_k(ri, rq, u);
            if (--rleft > 0) advance(ri, rq);
        };
        // D operands: FP64 [kind][bin quad]; BF16 [kind][MFMA]: the K halves of
        // MFMA m pair the limbs (D2 mu0 + D1 mu1), (D0 mu2 + D1 mu0),
        // (D0 mu1 + D0 mu0): A limb of this lane's half, (2, 0, 0) below lane
        // 32 and (1, 1, 0) above; mu limb (0, 2, 1) and (1, 0, 0)
        const int hk = lane >> 5;
        double A64[2][8];
        uint4 A16[2][6];
        auto load_a = [&](int ch, int set) {
            if (PREC == 0) {
                const double2 *at = (const double2 *)B.a64 + (long)ch * 4 * 64 + lane;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double2 v = at[u * 64];
                    A64[set][2 * u] = v.x;
                    A64[set][2 * u + 1] = v.y;
                }
            } else {
                const uint4 *at = B.a16 + (long)ch * 2 * 3 * 32 + (lane & 31);
                const int l0 = hk ? 1 : 2, l1 = hk ? 1 : 0;
#pragma unroll
                for (int kind = 0; kind < 2; ++kind) {
                    A16[set][3 * kind + 0] = at[(kind * 3 + l0) * 32];
                    A16[set][3 * kind + 1] = at[(kind * 3 + l1) * 32];
                    A16[set][3 * kind + 2] = at[(kind * 3 + 0) * 32];
                }
            }
        };
        auto step = [&](int ch, int u) {
            const int i = ci, q = cq;
            advance(ci, cq);
            load_a(ch + 1 < c1 ? ch + 1 : ch, (u + 1) & 1);
            if (q != colq) {
                flush_block(colq);
                colq = q;
                load_block(q);
            }
            const int wb = wbl[i];
            const double ni = nrow[i], mi = mk[i], qri = qrow[frow[i]];
            double Sc[4], Sf[4];
            if (PREC == 0) {
                f64x4 ac = {0.0, 0.0, 0.0, 0.0}, af = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double bm = murow[wb + 4 * t + g];
                    ac = __builtin_amdgcn_mfma_f64_16x16x4f64(A64[u & 1][t], bm, ac, 0, 0, 0);
                    af = __builtin_amdgcn_mfma_f64_16x16x4f64(A64[u & 1][4 + t], bm, af, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    Sc[r] = ac[r];
                    Sf[r] = af[r];
                }
            } else {
                float xs[8];
                const float *mrow = muf + cl * NS + wb + 8 * ((lane >> 4) & 1);
#pragma unroll
                for (int e = 0; e < 8; ++e) xs[e] = mrow[e];
                const Limbs8 U = split3x8(xs);
                const bf16x8 b0 = hk ? U.a1 : U.a0, b1 = hk ? U.a0 : U.a2, b2 = hk ? U.a0 : U.a1;
                union {
                    uint4 u;
                    bf16x8 v;
                } Ac[3], Af[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    Ac[m].u = A16[u & 1][m];
                    Af[m].u = A16[u & 1][3 + m];
                }
                f32x4 ac = {0.0f, 0.0f, 0.0f, 0.0f}, af = {0.0f, 0.0f, 0.0f, 0.0f};
                ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ac[0].v, b0, ac, 0, 0, 0);
                af = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Af[0].v, b0, af, 0, 0, 0);
                ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ac[1].v, b1, ac, 0, 0, 0);
                af = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Af[1].v, b1, af, 0, 0, 0);
                ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ac[2].v, b2, ac, 0, 0, 0);
                af = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Af[2].v, b2, af, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    Sc[r] = mus * (double)ac[r];
                    Sf[r] = mus * (double)af[r];
                }
            }
            double rows = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 16 * q + pj(r);
                const bool ok = j <= i;
                bool crater;
                const double fm = frag_mass(mi, mjr[r], chi, crater);
                const double qd = crater ? qcr[r] : qri;
                const double sc = Sc[r] - lmu[r];
                const double sf = (Sf[r] + fm * qd) - lmu[r];
                const double kf = (double)rf[u][r];
                const double ga = ok ? (double)rc[u][r] * sc + kf * sf : 0.0;
                const double aa = ok ? ni * njr[r] : 0.0;
                rows += njr[r] * ga;
                col[r] += ni * ga;
                const double D = aa * (double)ex[u][r] * kf * (sf - sc);
                gacc_a += (double)ez[u][r] * (aa * ga + D);
                if (VI) gacc_a += (double)ew[u][VI ? r : 0] * (aa * ga);
                gacc_v += D;
            }
            atomicAdd(&gnrow[i], rows);
            next_k(u);
        };
#pragma unroll
        for (int u = 0; u < kRingA; ++u) next_k(u);
        load_a(c0, 0);
        const int cend = c0 + (c1 - c0) / kRingA * kRingA;
        int ch = c0;
        for (; ch < cend; ch += kRingA) {
#pragma unroll
            for (int u = 0; u < kRingA; ++u) step(ch + u, u);
        }
#pragma unroll
        for (int u = 0; u < kRingA - 1; ++u)
            if (ch + u < c1) step(ch + u, u);
        flush_block(colq);
    };

    for (int t = 0; t < maxn; ++t) {
        for (int v = 3; v >= 1; --v) {
            prepare(wv, t, v);
            prepare(wv + 8, t, v);
            __syncthreads();
            contract();
            __syncthreads();
        }
    }
    // the last iteration's lambda += v1 (cells whose last step was in it)
    if (maxn > 0) {
        prepare(wv, maxn, 0);
        prepare(wv + 8, maxn, 0);
    }
    {
        const int cl = lane & 15;
        atomicAdd(&red[2 * cl], gacc_a);
        atomicAdd(&red[2 * cl + 1], gacc_v);
    }
    __syncthreads();
    for (int u = 0; u < 2; ++u) {
        const int c = wv + 8 * u;
        const long gc = cell0 + c;
        if (gc >= C) continue;
        const bool bad = ctl[c].bad;
        if (bad)
            for (int k = lane; k < N; k += 64) a.g_in[gc * N + k] = NAN;
        if (lane == 0) {
            const double vf = a.v_frag[gc];
            a.g_alpha[gc] = bad ? NAN : red[2 * c];
            a.g_vfrag[gc] = bad ? NAN : vf != 0.0 ? -red[2 * c + 1] / vf : 0.0;
        }
    }
}

template <typename K>
hipError_t allow_lds_a(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

}  // namespace

bool adj_batch_available(const Tables &T, const BatchTables &B) {
    return batch_available(T, B) && adj_lds_layout(T.N, 1).total <= 160 * 1024;
}

hipError_t launch_rate_derivs_blocked(const Tables &T, long C, const CellArrays &cells,
                                      const double *v_dust, const double *v_frag, int f32,
                                      void *Z, void *X, void *W, hipStream_t st) {
    if (C == 0) return hipSuccess;
    const bool vi = T.vertical != 0;
    if (vi && !W) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((C + 15) / 16);
    const unsigned slices = blocks >= 512 ? 1u : min(8u, (512u + blocks - 1) / blocks);
    const bool tab4 = (vi ? derivs_lds_bytes<4, true>(T.N) : derivs_lds_bytes<4, false>(T.N)) <=
                      160 * 1024;
#define DERIVS(TAB, VI, GT)                                                                     \
    {                                                                                           \
        const size_t bytes = derivs_lds_bytes<TAB, VI>(T.N);                                    \
        if (hipError_t e = allow_lds_a(k_rate_derivs_blk<TAB, VI, GT>, bytes)) return e;        \
        hipLaunchKernelGGL((k_rate_derivs_blk<TAB, VI, GT>), dim3(blocks, slices), dim3(1024),  \
                           bytes, st, T, cells, v_dust, v_frag, (GT *)Z, (GT *)X, (GT *)W, C);  \
    }
    if (!vi) {
        if (f32) {
            if (tab4) DERIVS(4, false, float) else DERIVS(1, false, float)
        } else {
            if (tab4) DERIVS(4, false, double) else DERIVS(1, false, double)
        }
    } else {
        if (f32) {
            if (tab4) DERIVS(4, true, float) else DERIVS(1, true, float)
        } else {
            if (tab4) DERIVS(4, true, double) else DERIVS(1, true, double)
        }
    }
#undef DERIVS
    return hipGetLastError();
}

hipError_t launch_adjoint_batch(const Tables &T, const BatchTables &B, long C,
                                const AdjBatchArgs &a, int prec, int gf32, hipStream_t st) {
    if (C == 0) return hipSuccess;
    if (!adj_batch_available(T, B)) return hipErrorNotSupported;
    const size_t bytes = adj_lds_layout(T.N, prec).total;
    const dim3 grid((unsigned)((C + kBC - 1) / kBC)), block(kBBlock);
    const bool vi = T.vertical != 0;
    if (vi && !a.W) return hipErrorInvalidValue;
#define LAUNCH(PR, RT, GT, VI)                                                                  \
    do {                                                                                        \
        if (hipError_t e = allow_lds_a(k_adj_batch<PR, RT, GT, VI>, bytes)) return e;          \
        hipLaunchKernelGGL((k_adj_batch<PR, RT, GT, VI>), grid, block, bytes, st, T, B, a, C); \
    } while (0)
    if (!vi) {
        if (prec == 0) LAUNCH(0, double, double, false);
        else if (gf32) LAUNCH(1, float, float, false);
        else LAUNCH(1, float, double, false);
    } else {
        if (prec == 0) LAUNCH(0, double, double, true);
        else if (gf32) LAUNCH(1, float, float, true);
        else LAUNCH(1, float, double, true);
    }
#undef LAUNCH
    return hipGetLastError();
}

}  // namespace coag
