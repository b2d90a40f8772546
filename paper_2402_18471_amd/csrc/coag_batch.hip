// coag_batch.hip -- cell-batched BS3(2) step with the gain contraction on the
// matrix cores.
//
// A workgroup (8 waves) advances a batch of 16 cells in lockstep: every
// right-hand side of eq. `smol` is evaluated for the 16 cells together, so
// that the gain sum G[cell, k] = sum_p R[cell, p] D[p, k] (R = n_i n_j K, D the
// fixed redistribution tensor of eqs. `Cijk`, `Rijk`) is a matrix product
// with the cells as its M dimension.  Pairs are taken in chunks of 16 of one
// row i (K = 32: the coagulating and the fragmenting rate of each pair); all
// coagulation and remnant products of row i land in a 16-bin window, the N
// dimension, together with bin i, which loses m_i per collision.  D, with that
// loss folded into its entries, is stored per chunk as MFMA B operands (FP64,
// or three BF16 limbs).
//
// What is not a matrix product stays on the vector units in FP64: the loss of
// the lighter grain m_j (a column sum), the fragment mass deposited at the top
// fragment bin (the accumulation of Rafikov et al. 2020, eq. `Nijk`), the
// fragment suffix sum, stage states, error control and the update.
//
// Split-BF16 form: the chunk operand A = n_j K / max_k n_k is formed in FP32
// and split into three BF16 limbs a0 + a1 + a2 (each the rounding of what the
// previous ones leave), D likewise; the six limb products of order <= 2 are
// accumulated in FP32 by v_mfma_f32_16x16x32_bf16 over one chunk and scaled
// back (x n_i max_k n_k) into the FP64 accumulators after every chunk.  The
// total mass of each cell is restored in FP64 at the end of the call.
//
// Cells of a batch that have finished (or lie past C) contribute zero rates
// and take no updates; the batch stops when every cell has.
#include <hip/hip_runtime.h>
#include <math.h>

#include "coag_batch.h"
#include "coag_batch_common.h"

namespace coag {

namespace {

using namespace bc;

// chunks of rates in flight per wave: the FP64 form has the registers for a
// deeper ring (one 8-wave workgroup per CU either way)
constexpr int kRing64 = 2, kRing16 = 2;
static_assert(kRing64 % 2 == 0 && kRing16 % 2 == 0,
              "the D operands alternate between two register sets by chunk parity");

// ---------------------------------------------------------------------------
// tables
// ---------------------------------------------------------------------------
int n_chunks(int N) {
    int nc = 0;
    for (int i = 0; i < N; ++i) nc += (i + 1 + 15) / 16;
    return nc;
}

// D entry of pair (i, j), kind (0 coagulation, 1 fragmentation), bin: the mass
// put into the bin per unit rate minus m_i for bin i (the heavier grain's
// loss).  Folding the loss into the entry keeps the near-cancellation of a
// heavy grain sweeping up a light one (gain into bin i ~ m_i) exact in FP64
// before any rounding to limbs.
__device__ double d_entry(const Tables &T, int i, int j, int kind, int bin) {
    if (j > i) return 0.0;
    const long p = (long)i * (i + 1) / 2 + j;
    const uint32_t d = T.dst[p];
    double v = 0.0;
    if (kind == 0) {
        const int c = d & 1023;
        if (bin == c) v += T.cw0[p];
        if (bin == c + 1) v += T.cw1[p];
    } else {
        const int r = (d >> 10) & 1023;
        if (bin == r) v += T.rw0[p];
        if (bin == r + 1) v += T.rw1[p];
    }
    if (bin == i) v -= T.m[i];
    return v;
}

// window of each row: the highest target minus 15, clipped to [0, N - 16]
__global__ void k_batch_rows(Tables T, int *wb, int *bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T.N) return;
    const int N = T.N;
    int lo = i, hi = i;
    for (int j = 0; j <= i; ++j) {
        const long p = (long)i * (i + 1) / 2 + j;
        const uint32_t d = T.dst[p];
        const int c = d & 1023, r = (d >> 10) & 1023;
        if (T.cw0[p] != 0.0) { lo = min(lo, c); hi = max(hi, c); }
        if (T.cw1[p] != 0.0) { lo = min(lo, c + 1); hi = max(hi, c + 1); }
        if (T.rw0[p] != 0.0) { lo = min(lo, r); hi = max(hi, r); }
        if (T.rw1[p] != 0.0) { lo = min(lo, r + 1); hi = max(hi, r + 1); }
    }
    int b = hi - (kWin - 1);
    if (b > N - kWin) b = N - kWin;
    if (b < 0) b = 0;
    wb[i] = b;
    if (lo < b || hi >= b + kWin) atomicOr(bad, 1);
}

// one thread per (chunk, lane): the B operands that lane holds for the chunk
__global__ void k_batch_b(Tables T, int NC, const int *crow, const int *crow_c, const int *wb,
                          double *b64, uint4 *b16) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)NC * 64) return;
    const int ch = (int)(t >> 6), lane = (int)(t & 63);
    int i = crow[ch] & 0xffff, q = crow[ch] >> 16;
    const int g = lane >> 4;
    int bin = wb[i] + (lane & 15);
    // FP64 operand of MFMA s: K row g <-> pair 16q + 4g + s % 4, kind s / 4
    for (int s = 0; s < 8; ++s)
        b64[(((long)ch * 4 + (s >> 1)) * 64 + lane) * 2 + (s & 1)] =
            d_entry(T, i, 16 * q + 4 * g + (s & 3), s >> 2, bin);
    // BF16 operand (chunks in the split form's order): K rows 8g + e <-> pair
    // 16q + 4g + e % 4, kind e / 4 (both kinds of four pairs in one lane)
    i = crow_c[ch] & 0xffff;
    q = crow_c[ch] >> 16;
    bin = wb[i] + (lane & 15);
    union {
        __bf16 h[8];
        uint4 u;
    } L0, L1, L2;
    for (int e = 0; e < 8; ++e) {
        const Limbs L = split3((float)d_entry(T, i, 16 * q + 4 * g + (e & 3), e >> 2, bin));
        L0.h[e] = L.a0;
        L1.h[e] = L.a1;
        L2.h[e] = L.a2;
    }
    b16[((long)ch * 3 + 0) * 64 + lane] = L0.u;
    b16[((long)ch * 3 + 1) * 64 + lane] = L1.u;
    b16[((long)ch * 3 + 2) * 64 + lane] = L2.u;
}

// one thread per (chunk, lane): the adjoint's A operands for the chunk
// (column-block order), pair 16q + l % 16 as the row.  FP64: bin quad t, bin
// wb + 4t + l / 16; BF16 (lanes 0..31): bins wb + 8 (l / 16) + e
__global__ void k_adj_a(Tables T, int NC, const int *crow_c, const int *wb, double *a64,
                        uint4 *a16) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)NC * 64) return;
    const int ch = (int)(t >> 6), lane = (int)(t & 63);
    const int i = crow_c[ch] & 0xffff, q = crow_c[ch] >> 16;
    const int j = 16 * q + (lane & 15);
    for (int kind = 0; kind < 2; ++kind)
        for (int tq = 0; tq < 4; ++tq) {
            const int e = kind * 4 + tq;            // operand e of the lane
            a64[(((long)ch * 4 + (e >> 1)) * 64 + lane) * 2 + (e & 1)] =
                d_entry(T, i, j, kind, wb[i] + 4 * tq + (lane >> 4));
        }
    if (lane >= 32) return;
    for (int kind = 0; kind < 2; ++kind) {
        union {
            __bf16 h[8];
            uint4 u;
        } L0, L1, L2;
        for (int e = 0; e < 8; ++e) {
            const Limbs L = split3((float)d_entry(T, i, j, kind, wb[i] + 8 * (lane >> 4) + e));
            L0.h[e] = L.a0;
            L1.h[e] = L.a1;
            L2.h[e] = L.a2;
        }
        uint4 *o = a16 + ((long)ch * 2 + kind) * 3 * 32 + lane;
        o[0] = L0.u;
        o[32] = L1.u;
        o[64] = L2.u;
    }
}

// ---------------------------------------------------------------------------
// per-cell control (one entry per cell of the batch, in LDS)
// ---------------------------------------------------------------------------
struct Ctl {
    double h, t, hh, mass0, atol, nmax, inv_nmax, fac;
    int nacc, nrej, status, nfix, clipped, active, live, pad;
};

template <int PREC, typename RT, bool BLK>
__global__ __launch_bounds__(kBBlock) void k_step_batch(Tables T, BatchTables B, StepArgs a,
                                                        long C, double *ws, RT *wk) {
    extern __shared__ double lds[];
    const int N = T.N;
    const long P = T.P;
    const long bt = batch_of(blockIdx.x, gridDim.x);
    const long cell0 = bt * kBC;
    // the per-cell rows of nv, net, phi and nf are NS = N | 1 elements apart:
    // an odd stride puts the same bin of the 16 cells, which a chunk's lanes
    // read and deposit together, in 16 different LDS banks for any N
    const int NS = batch_row_stride(N);
    double *nv = lds, *net = lds + kBC * NS, *phi = lds + 2 * kBC * NS, *mk = lds + 3 * kBC * NS;
    int *fcol = (int *)(mk + N), *frow = fcol + N, *wbl = frow + N;
    float *nf = (float *)(fcol + 4 * N);          // split form: [16][NS] n_k / max_k n_k
    Ctl *ctl = (Ctl *)(mk + 3 * N + kBC / 2 * NS);
    int *flag = (int *)(ctl + kBC);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int k = threadIdx.x; k < N; k += kBBlock) {
        mk[k] = T.m[k];
        fcol[k] = T.fcol[k];
        frow[k] = T.frow[k];
        wbl[k] = B.wb[k];
    }
    const bool adaptive = a.mode == 0;
    const double dt = a.dt;
    // workspace of cell c: k1, k2, k3, k4, yn, each [N]
    auto wsp = [&](int c, int v) { return ws + ((cell0 + c) * 5 + v) * (long)N; };

    // ---- FP64 form fed [C][P] rates: the batch's rates, reordered once per
    // call into the blocked layout of coag_rates_blocked (blk_elem), so that
    // every right-hand side streams whole cache lines (rows of [C][P] are P
    // elements apart).  Staged through LDS tiles of TP pairs (rows padded by
    // one element against bank conflicts).  Fed the blocked rates (BLK), both
    // forms read them in place, one 16-byte load per lane and pair (FP64) or
    // pair of pairs (FP32); the split form reads FP64 [C][P] rates directly.
    const long SL = pair_slot0(N);                  // pair slots per block
    RT *const kb = wk + bt * 64 * SL;
    if (PREC == 0 && !BLK) {
        RT *tile = (RT *)lds;
        const int cap = (int)((3 * kBC * N * sizeof(double)) / (2 * kBC * sizeof(RT))) - 1;
        const int TP = cap < 128 ? cap : 128, TS = TP + 1;
        const RT *src[2] = {(const RT *)a.Kc, (const RT *)a.Kf};
        for (long p0 = 0; p0 < P; p0 += TP) {
            const int np = P - p0 < TP ? (int)(P - p0) : TP;
            for (int t = threadIdx.x; t < 2 * kBC * TP; t += kBBlock) {
                const int pp = t % TP, r = t / TP;          // r = kind * 16 + cell
                const long gc = cell0 + (r & 15);
                tile[r * TS + pp] = (pp < np && gc < C) ? src[r >> 4][gc * P + p0 + pp] : (RT)0;
            }
            __syncthreads();
            for (int t = threadIdx.x; t < 2 * kBC * np; t += kBBlock) {
                const int kind = t & 1, c = (t >> 1) & 15, pp = t >> 5;
                const uint32_t ij = T.pij[p0 + pp];
                const int i = pair_i(ij), j = pair_j(ij);
                const long sl = pair_slot0(i) + (j >> 1);
                kb[blk_elem<RT>(sl, j & 1, c, kind)] = tile[(kind * 16 + c) * TS + pp];
                if (i == j && !(i & 1)) kb[blk_elem<RT>(sl, 1, c, kind)] = (RT)0;
            }
            __syncthreads();
        }
    }

    // ---- set-up: each wave owns cells wv and wv + 8 ----
    for (int u = 0; u < 2; ++u) {
        const int c = wv + 8 * u;
        const long gc = cell0 + c;
        const bool live = gc < C;
        double ms = 0.0;
        if (live)
            for (int k = lane; k < N; k += 64) ms += a.rho[gc * N + k];
        if (live && a.Ys)
            for (int k = lane; k < N; k += 64)
                a.Ys[gc * (a.max_sub + 1L) * N + k] = a.rho[gc * N + k];
        ms = wave_sum_d(ms);
        if (lane == 0) {
            Ctl &s = ctl[c];
            s.live = live;
            s.active = live;
            s.mass0 = ms;
            s.atol = a.atol_rel * ms;
            s.nacc = s.nrej = s.status = 0;
            s.nfix = 0;
            s.t = 0.0;
            s.hh = 0.0;
            s.clipped = 0;
            s.h = 0.0;
            if (live) {
                if (adaptive) {
                    s.h = a.h[gc] > 0.0 ? a.h[gc] : dt;
                } else {
                    s.nfix = a.nsub[gc];
                    if (s.nfix < 0 || s.nfix > a.max_sub) {
                        s.status = 2;
                        s.nfix = 0;
                    }
                }
            }
        }
    }
    __syncthreads();

    // ---- helpers ----
    // state of stage `stage` of cell c at bin k (0: y, 2, 3: stage states, 4: y+)
    auto form = [&](int stage) {
        for (int u = 0; u < 2; ++u) {
            const int c = wv + 8 * u;
            const long gc = cell0 + c;
            const bool on = stage == 0 ? ctl[c].live : ctl[c].active;
            double mx = 0.0;
            if (on) {
                const double hh = ctl[c].hh;
                const double *y = a.rho + gc * N;
                const double *k1 = wsp(c, 0), *k2 = wsp(c, 1), *k3 = wsp(c, 2);
                double *yn = wsp(c, 4);
                // REPLAY with kept stages: y2, y3 of sub-step nacc
                double *zs = a.Zs && (stage == 2 || stage == 3)
                                 ? a.Zs + ((gc * a.max_sub + ctl[c].nacc) * 2 + (stage - 2)) * (long)N
                                 : nullptr;
                for (int k = lane; k < N; k += 64) {
                    double x;
                    if (stage == 0) x = y[k];
                    else if (stage == 2) x = y[k] + 0.5 * hh * k1[k];
                    else if (stage == 3) x = y[k] + 0.75 * hh * k2[k];
                    else {
                        x = y[k] + hh * (2.0 / 9.0 * k1[k] + 1.0 / 3.0 * k2[k] + 4.0 / 9.0 * k3[k]);
                        yn[k] = x;
                    }
                    if (zs) zs[k] = x;
                    const double n = x / mk[k];
                    nv[c * NS + k] = n;
                    mx = fmax(mx, fabs(n));
                }
            } else {
                for (int k = lane; k < N; k += 64) nv[c * NS + k] = 0.0;
            }
            for (int k = lane; k < N; k += 64) {
                net[c * NS + k] = 0.0;
                phi[c * NS + k] = 0.0;
            }
            if (PREC == 1) {
                mx = wave_max_d(mx);
                const double inv = mx > 0.0 ? 1.0 / mx : 0.0;
                for (int k = lane; k < N; k += 64) nf[c * NS + k] = (float)(nv[c * NS + k] * inv);
                if (lane == 0) {
                    ctl[c].nmax = mx;
                    ctl[c].inv_nmax = inv;
                }
            }
        }
    };

    // ---- FP64 form: gain and loss of all 16 cells into net (gain - loss
    // without the fragment distribution) and phi (fragment mass per top bin).
    // Chunks in row-major order, each wave a contiguous range of them: the
    // gain tile of a row accumulates over the row's chunks and is deposited
    // when the row changes; the loss of the lighter grain and the fragment mass
    // are deposited per pair.  The rates, the one stream from HBM, are loaded
    // kRing64 chunks ahead into a register ring, the D operands one chunk ahead.
    // Every chunk issues the same loads in the same order, past the wave's
    // last chunk repeating it, so that they are unconditional and each operand
    // is waited for only when it is used.
    auto contract64 = [&]() {
        const int cl = lane & 15, g = lane >> 4;
        const int NC = B.NC;
        const int c0 = (int)((long)wv * NC / kBWaves), c1 = (int)((long)(wv + 1) * NC / kBWaves);
        if (c0 >= c1) return;
        const double *nrow = nv + cl * NS;
        double *netc = net + cl * NS, *phic = phi + cl * NS;
        const double chi = T.chi;
        // (i, q) -> (i, q + 1) or (i + 1, 0)
        auto advance = [](int &i, int &q) {
            if (16 * (q + 1) <= i) ++q;
            else { ++i; q = 0; }
        };
        const int cr0 = __builtin_amdgcn_readfirstlane(B.crow[c0]);
        int ci = cr0 & 0xffff, cq = cr0 >> 16;     // chunk being processed
        int ri = ci, rq = cq;                       // next chunk to load rates for
        int cur = ci;
        // two accumulators, coagulating and fragmenting products, so that the
        // chunk's matrix products form two dependent chains of four, not one
        // of eight
        f64x4 acc64 = {0.0, 0.0, 0.0, 0.0}, acf64 = {0.0, 0.0, 0.0, 0.0};
        // accumulator layout of v_mfma_f64_16x16x4f64: lane l, register r ->
        // row (cell) l / 16 + 4 r, column (bin) l % 16
        auto flush = [&](int i) {
            const int bin = wbl[i] + cl;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                atomicAdd(&net[(g + 4 * r) * NS + bin], acc64[r] + acf64[r]);
        };
        // the batch's rates: reordered in the workspace, or the caller's
        // blocked array, both in the blocked layout, read through a raw buffer
        // over the batch (byte offsets below 2^32 for N <= 1023)
        const RT *kbb = BLK ? (const RT *)a.Kc + cell0 / kBC * 64 * SL : kb;
        const __amdgpu_buffer_rsrc_t kr = raw_buffer(kbb, (unsigned)(64 * SL * sizeof(RT)));
        // lane (cell, g): pairs 16q + 4g + s, s = 0..3, both kinds
        double rkc[kRing64][4], rkf[kRing64][4], bb[2][8];
        auto load_k = [&](int i, int q, double (&kc)[4], double (&kf)[4]) {
            const unsigned s0 = (unsigned)pair_slot0(i);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int j = 16 * q + 4 * g + s, jc = j <= i ? j : i;
                const unsigned o = (unsigned)blk_elem<double>(s0 + (jc >> 1), jc & 1, cl, 0) * 8u;
                // streaming loads: the rates are read once per right-hand
                // side, and keeping them out of L2 leaves it to the D
                // operands every batch shares (9 % less traffic, 2 % faster)
                const f64x2 v = buf_f64x2<true>(kr, o);
                kc[s] = v[0];
                kf[s] = v[1];
            }
        };
        // the chunk's eight operands of this lane as four 16-byte loads, each
        // contiguous over the wave
        auto load_b = [&](int ch, double (&b)[8]) {
            const double2 *bt = (const double2 *)B.b64 + (long)ch * 4 * 64 + lane;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double2 v = bt[u * 64];
                b[2 * u] = v.x;
                b[2 * u + 1] = v.y;
            }
        };
        int rleft = c1 - c0;                        // chunks whose rates are still to load
        auto next_k = [&](double (&kc)[4], double (&kf)[4]) {
            load_k(ri, rq, kc, kf);
            if (--rleft > 0) advance(ri, rq);
        };
        // the heavier grain's values, per row
        double ni = nrow[cur], mi = mk[cur];
        int fri = frow[cur];
        // One chunk.  The lane's four pairs read all their LDS operands first
        // and deposit their column terms (loss of the lighter grain, fragment
        // mass at its top bin) last, so that no read waits behind an atomic.
        auto step = [&](int ch, int u) {
            const int i = ci, q = cq;
            advance(ci, cq);
            load_b(ch + 1 < c1 ? ch + 1 : ch, bb[(u + 1) & 1]);
            if (i != cur) {
                flush(cur);
                cur = i;
                acc64 = f64x4{0.0, 0.0, 0.0, 0.0};
                acf64 = f64x4{0.0, 0.0, 0.0, 0.0};
                ni = nrow[i];
                mi = mk[i];
                fri = frow[i];
            }
            int jc[4], fc[4];
            bool ok[4];
            double nj[4], mj[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int j = 16 * q + 4 * g + s;
                ok[s] = j <= i;
                jc[s] = ok[s] ? j : i;
                nj[s] = nrow[jc[s]];
                mj[s] = mk[jc[s]];
                fc[s] = fcol[jc[s]];
            }
            double rc[4], rf[4], loss[4], frag[4];
            int fdst[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double nn = ok[s] ? ni * nj[s] : 0.0;
                rc[s] = nn * rkc[u][s];
                rf[s] = nn * rkf[u][s];
                loss[s] = -mj[s] * (rc[s] + rf[s]);
                bool crater;
                frag[s] = frag_mass(mi, mj[s], chi, crater) * rf[s];
                fdst[s] = crater ? fc[s] : fri;
            }
            const double(&b)[8] = bb[u & 1];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc64 = __builtin_amdgcn_mfma_f64_16x16x4f64(rc[s], b[s], acc64, 0, 0, 0);
                acf64 = __builtin_amdgcn_mfma_f64_16x16x4f64(rf[s], b[4 + s], acf64, 0, 0, 0);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                atomicAdd(&netc[jc[s]], loss[s]);
                atomicAdd(&phic[fdst[s]], frag[s]);
            }
            next_k(rkc[u], rkf[u]);
        };
#pragma unroll
        for (int u = 0; u < kRing64; ++u) next_k(rkc[u], rkf[u]);
        load_b(c0, bb[0]);
        const int cend = c0 + (c1 - c0) / kRing64 * kRing64;
        int ch = c0;
        for (; ch < cend; ch += kRing64) {
#pragma unroll
            for (int u = 0; u < kRing64; ++u) step(ch + u, u);
        }
#pragma unroll
        for (int u = 0; u < kRing64 - 1; ++u)
            if (ch + u < c1) step(ch + u, u);
        flush(cur);
    };

    // ---- split form: the same terms, chunks taken column block by column
    // block (q outer, row i inner), each wave a contiguous range of them, so a
    // lane keeps the same lighter grains j over many chunks: the loss of grain
    // j (m_j times the sum of its rates) and the crater fragments (all at the
    // top bin of j) are summed in registers and deposited when the column
    // block changes.  The FP32 gain tile of a chunk (row i's window) is scaled
    // back and deposited while the next chunk's products run.  Rates are
    // loaded kRing16 chunks ahead into a register ring, D operands one ahead,
    // unconditionally as in the FP64 form.
    auto contract16 = [&]() {
        const int cl = lane & 15, g = lane >> 4;
        const int NC = B.NC;
        const int c0 = (int)((long)wv * NC / kBWaves), c1 = (int)((long)(wv + 1) * NC / kBWaves);
        if (c0 >= c1) return;
        const double *nrow = nv + cl * NS;
        double *netc = net + cl * NS, *phic = phi + cl * NS;
        const double nmax = ctl[cl].nmax;
        const float *nfr = nf + cl * NS;
        const double chi = T.chi;
        // (i, q) -> (i + 1, q), or the top of the next column block
        auto advance = [N](int &i, int &q) {
            if (i + 1 < N) ++i;
            else { ++q; i = 16 * q; }
        };
        const int cr0 = __builtin_amdgcn_readfirstlane(B.crow_c[c0]);
        int ci = cr0 & 0xffff, cq = cr0 >> 16;     // chunk being processed
        int ri = ci, rq = cq;                       // next chunk to load rates for
        // two tiles, used by alternate chunks: a chunk's tile is deposited
        // after the next chunk's products have been issued into the other one
        f32x4 acc32[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
        // accumulator layout of v_mfma_f32_16x16x32_bf16: lane l, register r ->
        // row (cell) 4 (l / 16) + r, column (bin) l % 16
        double tmax[4];                             // max n of the tile's cells 4g + r
#pragma unroll
        for (int r = 0; r < 4; ++r) tmax[r] = ctl[4 * g + r].nmax;
        auto flush_tile = [&](int i, int t) {
            const int bin = wbl[i] + cl;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = 4 * g + r;
                const double f = nv[c * NS + i] * tmax[r];
                atomicAdd(&net[c * NS + bin], f * (double)acc32[t][r]);
            }
            acc32[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        };
        // this lane's lighter grains in column block q (both kinds of four
        // pairs), and their running sums: all rates of grain j, and its
        // fragmenting rates against the targets it craters.  A cratering
        // projectile j makes fragments of mass (1 + chi) m_j (itself and the
        // mass it excavates, eq. `fragrem`), all at the top bin of j, so the
        // factor is applied once per block.
        constexpr int NJ = 4;
        auto jof = [&](int q, int u) { return 16 * q + 4 * g + u; };
        // The sums restart with the first chunk of each block, which scales
        // them by keep = 0 as it adds its own terms (later chunks: keep = 1),
        // rather than clearing them in the branch that deposits them.
        double colsum[NJ], cratsum[NJ];
#pragma unroll
        for (int u = 0; u < NJ; ++u) colsum[u] = cratsum[u] = 0.0;
        auto flush_cols = [&](int q) {
#pragma unroll
            for (int u = 0; u < NJ; ++u) {
                const int j = jof(q, u);
                if (j < N) {
                    const double mj = mk[j];
                    atomicAdd(&netc[j], -mj * colsum[u]);
                    atomicAdd(&phic[fcol[j]], (1.0 + chi) * mj * cratsum[u]);
                }
            }
        };
        // n_j / max n of the lane's four lighter grains (zero past the grid)
        // and chi m_j of the block's heaviest: constant over a column block
        float njv[NJ];
        double mq = 0.0;
        auto load_cols = [&](int q) {
#pragma unroll
            for (int u = 0; u < NJ; ++u) {
                const int j = jof(q, u);
                njv[u] = j < N ? nfr[j] : 0.0f;
            }
            mq = chi * mk[16 * q + 15 < N ? 16 * q + 15 : N - 1];
        };
        int colq = cq, prev = -1;
        load_cols(colq);
        // lane (cell, g): pairs 16q + 4g + s, s = 0..3, Kc in k[s], Kf in
        // k[4 + s] (the K rows of the MFMA operands)
        // FP32 rates: pair p of the batch's cell cl at p * 16 + cl (padding
        // cells hold zeros); FP64 rates: [C][P], cells past C read cell C - 1
        constexpr bool blk = BLK;
        const long cb = cell0 + cl < C ? cell0 + cl : C - 1;
        // blocked rates: the batch's uniform base and 32-bit lane offsets
        // (pair p of cell cl at p * 16 + cl); [C][P] rates: the lane's cell
        // blocked FP32 rates: the batch's block of the caller's array (two
        // pairs, both kinds, per 16-byte load); [C][P] FP64 rates: from the
        // batch's first cell, cell cl at (cb - cell0) * P + p (cells past C
        // read cell C - 1).  Byte offsets below 2^32 for N <= 1023.
        const long SL = pair_slot0(N);
        const unsigned kl = (unsigned)((cb - cell0) * P);
        const RT *Kc = (const RT *)a.Kc + (blk ? cell0 / kBC * 64 * SL : cell0 * P);
        const RT *Kf = blk ? Kc : (const RT *)a.Kf + cell0 * P;
        const long ncb = C - cell0 < kBC ? C - cell0 : kBC;
        const unsigned span = (unsigned)((blk ? 64 * SL : ncb * P) * sizeof(RT));
        const __amdgpu_buffer_rsrc_t kcr = raw_buffer(Kc, span), kfr = raw_buffer(Kf, span);
        RT rk[kRing16][8];
        uint4 bb[2][3];
        auto load_k = [&](int i, int q, RT (&k)[8]) {
            if constexpr (blk) {
                // pairs 4g + 2u, 4g + 2u + 1 (clamped to the row's last slot:
                // pairs past the diagonal are masked where they are used)
                const unsigned s0 = (unsigned)pair_slot0(i);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int j = 16 * q + 4 * g + 2 * u, jc = j <= i ? j : i;
                    const unsigned o = (unsigned)blk_elem<float>(s0 + (jc >> 1), 0, cl, 0) * 4u;
                    const f32x4 v = buf_f32x4<false>(kcr, o);
                    k[2 * u] = v[0];
                    k[4 + 2 * u] = v[1];
                    k[2 * u + 1] = v[2];
                    k[5 + 2 * u] = v[3];
                }
            } else {
                const unsigned prow = (unsigned)(i * (i + 1) / 2);
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int j = 16 * q + 4 * g + s;
                    const unsigned o = (prow + (unsigned)(j <= i ? j : i) + kl) * 8u;
                    k[s] = buf_f64<false>(kcr, o);
                    k[4 + s] = buf_f64<false>(kfr, o);
                }
            }
        };
        auto load_b = [&](int ch, uint4 (&b)[3]) {
            const uint4 *bt = B.b16 + (long)ch * 3 * 64 + lane;
            b[0] = bt[0];
            b[1] = bt[64];
            b[2] = bt[128];
        };
        int rleft = c1 - c0;                        // chunks whose rates are still to load
        auto next_k = [&](RT (&k)[8]) {
            load_k(ri, rq, k);
            if (--rleft > 0) advance(ri, rq);
        };
        auto step = [&](int ch, int u) {
            const int i = ci, q = cq;
            advance(ci, cq);
            load_b(ch + 1 < c1 ? ch + 1 : ch, bb[(u + 1) & 1]);
            const bool fresh = q != colq;
            if (fresh) {
                flush_cols(colq);
                colq = q;
                load_cols(q);
            }
            const double keep = fresh ? 0.0 : 1.0;
            // x = n_j K / max n (FP32, the MFMA operand); the FP64 rate of
            // the pair for the column terms is (n_i max n) x.  Column terms:
            // the rate sums, and fragments (crater: summed for the block;
            // destroyed target, mass m_i + m_j: summed for the chunk, all at
            // the top bin of m_i).  Grain i craters every grain of the block
            // when it craters the heaviest (chi m_j < m_i), the case of all
            // but the chunks near the diagonal.
            const double c64 = nrow[i] * nmax, mi = mk[i];
            float x[8];
            double dest = 0.0;
            auto pairs = [&](bool full, bool crat) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int j = 16 * q + 4 * g + s;
                    const bool ok = full || j <= i;
                    const int jc = ok ? j : i;
                    x[s] = ok ? njv[s] * (float)rk[u][s] : 0.0f;
                    x[4 + s] = ok ? njv[s] * (float)rk[u][4 + s] : 0.0f;
                    const double xf = (double)x[4 + s];
                    colsum[s] = fma(colsum[s], keep, c64 * ((double)x[s] + xf));
                    const double rf = c64 * xf;
                    if (crat) {
                        cratsum[s] = fma(cratsum[s], keep, rf);
                    } else {
                        const double mj = mk[jc];
                        const bool crater = chi * mj < mi;
                        cratsum[s] = fma(cratsum[s], keep, crater ? rf : 0.0);
                        dest += crater ? 0.0 : (mi + mj) * rf;
                    }
                }
            };
            if (16 * q + 15 <= i && mq < mi) {
                pairs(true, true);
            } else {
                if (16 * q + 15 <= i) pairs(true, false);
                else pairs(false, false);
                atomicAdd(&phic[frow[i]], dest);
            }
            const Limbs8 L = split3x8(x);
            union {
                uint4 u;
                bf16x8 v;
            } B0, B1, B2;
            B0.u = bb[u & 1][0];
            B1.u = bb[u & 1][1];
            B2.u = bb[u & 1][2];
            // one chunk per FP32 accumulation, the limb products smallest
            // first (order 2, 1, 0): each MFMA rounds its sum to FP32 once, so
            // the corrections are summed before they meet the a0 b0 term
            f32x4 &acc = acc32[u & 1];
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L.a2, B0.v, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L.a1, B1.v, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L.a0, B2.v, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L.a1, B0.v, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L.a0, B1.v, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L.a0, B0.v, acc, 0, 0, 0);
            if (prev >= 0) flush_tile(prev, (u + 1) & 1);
            prev = i;
            next_k(rk[u]);
        };
#pragma unroll
        for (int u = 0; u < kRing16; ++u) next_k(rk[u]);
        load_b(c0, bb[0]);
        const int cend = c0 + (c1 - c0) / kRing16 * kRing16;
        int ch = c0;
        for (; ch < cend; ch += kRing16) {
#pragma unroll
            for (int u = 0; u < kRing16; ++u) step(ch + u, u);
        }
#pragma unroll
        for (int u = 0; u < kRing16 - 1; ++u)
            if (ch + u < c1) step(ch + u, u);
        flush_tile(prev, (c1 - 1 - c0) & 1);        // the last chunk's tile
        flush_cols(colq);
    };

    auto contract = [&]() {
        if (PREC == 0) contract64();
        else contract16();
    };

    // slope of cell c: net + dE_k sum_{l >= k} phi_l invE_l, into ws slot v
    auto finish = [&](int stage, int v) {
        for (int u = 0; u < 2; ++u) {
            const int c = wv + 8 * u;
            const bool on = stage == 0 ? ctl[c].live : ctl[c].active;
            if (!on) continue;
            double *out = wsp(c, v);
            double carry = 0.0;
            for (int top = N - 1; top >= 0; top -= 64) {
                const int k = top - lane;
                double x = k >= 0 ? phi[c * NS + k] * T.invE[k] : 0.0;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const double y = __shfl_up(x, o, 64);
                    if (lane >= o) x += y;
                }
                if (k >= 0) out[k] = net[c * NS + k] + T.dE[k] * (x + carry);
                carry += __shfl(x, 63, 64);
            }
        }
    };

    // set up the next attempt of cell c (owner wave, after a block barrier)
    auto begin = [&](int c) {
        Ctl &s = ctl[c];
        if (!s.active) return;
        bool go = true;
        if (adaptive) {
            if (!(s.t < dt)) go = false;
            else if (s.nacc + s.nrej >= a.max_sub) { s.status = 2; go = false; }
            else {
                s.hh = s.h;
                s.clipped = 0;
                if (s.hh >= dt - s.t) { s.hh = dt - s.t; s.clipped = 1; }
                if (!s.clipped && s.hh < a.h_min_rel * dt) { s.status = 1; go = false; }
            }
        } else {
            if (s.nacc >= s.nfix) go = false;
            else s.hh = a.mode == 1 ? dt / s.nfix : a.h_log[(cell0 + c) * (long)a.max_sub + s.nacc];
        }
        s.active = go;
    };

    // accept / reject the attempt of cell c (owner wave)
    auto decide = [&](int c) {
        Ctl &s = ctl[c];
        if (!s.active) return;
        const long gc = cell0 + c;
        double *y = a.rho + gc * N;
        const double *k1 = wsp(c, 0), *k2 = wsp(c, 1), *k3 = wsp(c, 2), *k4 = wsp(c, 3),
                     *yn = wsp(c, 4);
        bool accept = true;
        double fac = 1.0;
        const double hh = s.hh;
        if (adaptive) {
            double qmax = 0.0, ymin = INFINITY, bad = 0.0;
            for (int k = lane; k < N; k += 64) {
                const double e = hh * (-5.0 / 72.0 * k1[k] + 1.0 / 12.0 * k2[k] + 1.0 / 9.0 * k3[k] -
                                       1.0 / 8.0 * k4[k]);
                const double sc = s.atol + a.rtol * fmax(fabs(y[k]), fabs(yn[k]));
                if (!isfinite(yn[k]) || !isfinite(e)) bad += 1.0;
                qmax = fmax(qmax, fabs(e) / sc);
                ymin = fmin(ymin, yn[k]);
            }
            bad = wave_sum_d(bad);
            const double err = wave_max_d(qmax);
            const double ylo = wave_min_d(ymin);
            if (bad > 0.0 || !isfinite(err)) {
                if (lane == 0) {
                    s.status = 3;
                    s.active = 0;
                }
                return;
            }
            fac = err == 0.0 ? 5.0 : 0.9 * pow(err, -1.0 / 3.0);
            fac = fmin(5.0, fmax(0.2, fac));
            accept = err <= 1.0 && !(ylo < -s.atol);
            if (!accept && lane == 0) s.h = hh * (err <= 1.0 ? 0.5 : fac);
        }
        if (accept) {
            for (int k = lane; k < N; k += 64) y[k] = yn[k];
            if (a.Ys) {
                double *ys = a.Ys + (gc * (a.max_sub + 1L) + s.nacc + 1) * N;
                for (int k = lane; k < N; k += 64) ys[k] = yn[k];
            }
            double *k1w = wsp(c, 0);
            for (int k = lane; k < N; k += 64) k1w[k] = k4[k];
            if (lane == 0) {
                if (a.h_log && s.nacc < a.max_sub && a.mode != 2)
                    a.h_log[gc * (long)a.max_sub + s.nacc] = hh;
                ++s.nacc;
                if (adaptive) {
                    s.t = s.clipped ? dt : s.t + hh;
                    if (!s.clipped) s.h = hh * fac;
                }
            }
        } else if (lane == 0) {
            ++s.nrej;
        }
    };

    // ---- the stage loop: 0 (k1 = f(y)), then 2, 3, 4 per attempt ----
    int stage = 0;
    while (true) {
        form(stage);
        __syncthreads();
        contract();
        __syncthreads();
        finish(stage, stage == 0 ? 0 : stage - 1);
        __syncthreads();
        if (stage == 0 || stage == 4) {
            if (stage == 4) {
                decide(wv);
                decide(wv + 8);
                __syncthreads();
            }
            if (threadIdx.x == 0) *flag = 0;
            __syncthreads();
            if (lane == 0) {
                begin(wv);
                begin(wv + 8);
                if (ctl[wv].active || ctl[wv + 8].active) atomicOr(flag, 1);
            }
            __syncthreads();
            if (!*flag) break;
            stage = 2;
        } else {
            ++stage;
        }
    }

    // ---- outputs; FP64 mass bookkeeping ----
    for (int u = 0; u < 2; ++u) {
        const int c = wv + 8 * u;
        Ctl &s = ctl[c];
        if (!s.live) continue;
        const long gc = cell0 + c;
        double *y = a.rho + gc * N;
        if (!adaptive && s.status == 0) {
            double bad = 0.0;
            for (int k = lane; k < N; k += 64) bad += isfinite(y[k]) ? 0.0 : 1.0;
            if (wave_sum_d(bad) > 0.0 && lane == 0) s.status = 3;
        }
        if ((a.renorm || PREC == 1) && s.status == 0) {
            double ms = 0.0;
            for (int k = lane; k < N; k += 64) ms += y[k];
            const double m1 = wave_sum_d(ms);
            if (m1 > 0.0) {
                const double sc = s.mass0 / m1;
                for (int k = lane; k < N; k += 64) y[k] *= sc;
            }
        }
        if (lane == 0) {
            if (adaptive) {
                a.h[gc] = s.h;
                a.nsub[gc] = s.nacc;
            }
            if (a.nrej) a.nrej[gc] = s.nrej;
            a.status[gc] = s.status;
        }
    }
}

size_t batch_lds_bytes(int N) {
    return ((size_t)(3 * kBC + kBC / 2) * batch_row_stride(N) + 3 * N) * sizeof(double) +
           kBC * sizeof(Ctl) + 64;
}

template <typename K>
hipError_t allow_lds_b(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

}  // namespace

size_t batch_tables_bytes(int N) {
    const size_t NC = (size_t)n_chunks(N);
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    return 2 * al(4 * NC) + al(4 * (size_t)N) + al(8 * NC * 8 * 64) + al(16 * NC * 3 * 64) +
           al(8 * NC * 2 * 4 * 64) + al(16 * NC * 2 * 3 * 32) + 256;
}

hipError_t build_batch_tables(const Tables &T, void *mem, BatchTables *B) {
    const int N = T.N;
    const int NC = n_chunks(N);
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    char *p = (char *)mem;
    int *crow = (int *)p;
    p += al(4 * (size_t)NC);
    int *crow_c = (int *)p;
    p += al(4 * (size_t)NC);
    int *wb = (int *)p;
    p += al(4 * (size_t)N);
    double *b64 = (double *)p;
    p += al(8 * (size_t)NC * 8 * 64);
    uint4 *b16 = (uint4 *)p;
    p += al(16 * (size_t)NC * 3 * 64);
    double *a64 = (double *)p;
    p += al(8 * (size_t)NC * 2 * 4 * 64);
    uint4 *a16 = (uint4 *)p;
    p += al(16 * (size_t)NC * 2 * 3 * 32);
    int *bad = (int *)p;
    B->NC = NC;
    B->ok = 0;
    B->crow = crow;
    B->crow_c = crow_c;
    B->wb = wb;
    B->b64 = b64;
    B->b16 = b16;
    B->a64 = a64;
    B->a16 = a16;
    if (N < kWin) return hipSuccess;                 // window wider than the grid: path off
    int *h = (int *)malloc(sizeof(int) * NC);
    if (!h) return hipErrorOutOfMemory;
    int c = 0;                                       // row by row (FP64 form)
    for (int i = 0; i < N; ++i)
        for (int q = 0; q * 16 <= i; ++q) h[c++] = i | (q << 16);
    hipError_t e = hipMemcpy(crow, h, sizeof(int) * NC, hipMemcpyHostToDevice);
    c = 0;                                           // column block by column block (split)
    for (int q = 0; 16 * q < N; ++q)
        for (int i = 16 * q; i < N; ++i) h[c++] = i | (q << 16);
    if (e == hipSuccess) e = hipMemcpy(crow_c, h, sizeof(int) * NC, hipMemcpyHostToDevice);
    free(h);
    if (e == hipSuccess) e = hipMemset(bad, 0, sizeof(int));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_rows, dim3((N + 63) / 64), dim3(64), 0, 0, T, wb, bad);
    hipLaunchKernelGGL(k_batch_b, dim3((unsigned)((NC * 64L + 255) / 256)), dim3(256), 0, 0, T, NC,
                       crow, crow_c, wb, b64, b16);
    hipLaunchKernelGGL(k_adj_a, dim3((unsigned)((NC * 64L + 255) / 256)), dim3(256), 0, 0, T, NC,
                       crow_c, wb, a64, a16);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int hb = 1;
    if ((e = hipMemcpy(&hb, bad, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess) return e;
    B->ok = hb == 0;
    return hipSuccess;
}

bool batch_available(const Tables &T, const BatchTables &B) {
    return B.ok && batch_lds_bytes(T.N) <= 160 * 1024;
}

static size_t slope_bytes(int N, long C) {
    const long nb = (C + kBC - 1) / kBC;
    return ((size_t)nb * kBC * 5 * N * sizeof(double) + 255) & ~size_t(255);
}

size_t batch_ws_bytes(int N, long C, int prec, int layout) {
    const long nb = (C + kBC - 1) / kBC;
    const bool reorder = prec == 0 && layout == 0;
    return slope_bytes(N, C) + (reorder ? (size_t)nb * 64 * pair_slot0(N) * sizeof(double) : 0);
}

hipError_t launch_step_batch(const Tables &T, const BatchTables &B, long C, const StepArgs &a,
                             int prec, int layout, double *ws, hipStream_t st, void *wk) {
    if (C == 0) return hipSuccess;
    if (!batch_available(T, B)) return hipErrorNotSupported;
    const size_t bytes = batch_lds_bytes(T.N);
    const dim3 grid((unsigned)((C + kBC - 1) / kBC)), block(kBBlock);
    char *wkp = wk ? (char *)wk : (char *)ws + slope_bytes(T.N, C);
#define LAUNCH(PR, RT, BL)                                                                   \
    do {                                                                                     \
        if (hipError_t e = allow_lds_b(k_step_batch<PR, RT, BL>, bytes)) return e;          \
        hipLaunchKernelGGL((k_step_batch<PR, RT, BL>), grid, block, bytes, st, T, B, a, C,  \
                           ws, (RT *)wkp);                                                   \
    } while (0)
    if (prec == 0 && layout == 0) LAUNCH(0, double, false);
    else if (prec == 0 && layout == 2) LAUNCH(0, double, true);
    else if (prec == 1 && layout == 0) LAUNCH(1, double, false);
    else if (prec == 1 && layout == 1) LAUNCH(1, float, true);
    else return hipErrorNotSupported;
#undef LAUNCH
    return hipGetLastError();
}

}  // namespace coag
