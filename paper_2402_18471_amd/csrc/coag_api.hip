// coag_api.hip -- the C ABI of libcoag (declared in include/coag.h): argument
// validation on the host, context lifetime, workspaces and kernel launches.
// Every numerical step of the path runs in the kernels of coag_kernels.hip,
// coag_step2.hip, coag_batch.hip and coag_adjoint.hip; this file only checks, allocates and
// launches.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>

#include "../../include/coag.h"
#include "coag_launch.h"
#include "coag_batch.h"

using namespace coag;

// Scratch of coag_step_noalloc: the batched step's workspace (slopes and stage
// states of every cell, and the reordered rates of [C][P] FP64 input) for
// callers that cannot allocate.  Each device holds its own copy, from the
// library's load to the end of the process; host code uses only the device
// address looked up per device at coag_create (g_scratch), never the name.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

struct coag_ctx {
    int device = -1;
    int N = 0, P = 0;
    double rho_m = 0, eta = 0, chi = 0;
    int split = 0;
    // device tables
    void *block = nullptr;                 // one allocation holding every table
    Tables T{};
    BatchTables B{};
    bool batch_fp64 = true;                // FP64 steps take the batched kernel when it applies
    long adj_slab = 0;                     // cells per slab of the batched adjoint (0: by budget)
    void *scratch = nullptr;               // this device's scratch array (coag_step_noalloc)
    // grow-only workspaces
    void *ws = nullptr;
    size_t ws_bytes = 0;
    std::string err;
};

static thread_local std::string g_err;

static int fail(coag_ctx *ctx, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    g_err = buf;
    return code;
}

#define HIP_TRY(ctx, call)                                                               \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ctx, COAG_EHIP, "%s: %s", #call, hipGetErrorString(e_));         \
    } while (0)

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static int ensure_ws(coag_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return COAG_OK;
    if (ctx->ws) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    if (hipMalloc(&ctx->ws, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, COAG_ENOMEM, "workspace allocation of %zu bytes failed", bytes);
    }
    ctx->ws_bytes = bytes;
    return COAG_OK;
}

static int set_device(coag_ctx *ctx) {
    int cur = -1;
    HIP_TRY(ctx, hipGetDevice(&cur));
    if (cur != ctx->device) HIP_TRY(ctx, hipSetDevice(ctx->device));
    return COAG_OK;
}

// the bin count of a context, for the transport scheduler (coag_transport.hip)
namespace coag {
int ctx_bins(const ::coag_ctx *ctx) { return ctx->N; }
// whether coag_step takes 16-cell-blocked rates in this precision (0 FP64,
// 1 split): the batched step applies to the grid, and for FP64 is selected
bool ctx_blocked(const ::coag_ctx *ctx, int prec) {
    return batch_available(ctx->T, ctx->B) && (prec == 1 || ctx->batch_fp64);
}
// whether the context takes the vertically integrated kernel
bool ctx_vertical(const ::coag_ctx *ctx) { return ctx->T.vertical != 0; }
}  // namespace coag

extern "C" {

int coag_mass_grid(int32_t n_bins, double lo, double hi, int32_t by_mass, double rho_m,
                   double *m, double *m_edge, double *s) {
    if (n_bins < 2 || !(lo > 0.0) || !(hi > lo) || !(rho_m > 0.0) || !m || !m_edge || !s)
        return fail(nullptr, COAG_EINVAL, "coag_mass_grid: need N >= 2, 0 < lo < hi, rho_m > 0 "
                                          "and non-null outputs");
    const int N = n_bins;
    auto mass = [&](double x) { return by_mass ? x : 4.0 * M_PI / 3.0 * rho_m * x * x * x; };
    for (int k = 0; k <= N; ++k) m_edge[k] = mass(lo * pow(hi / lo, (double)k / (double)N));
    for (int k = 0; k < N; ++k) {
        const double x = lo * pow(hi / lo, (k + 0.5) / (double)N);
        m[k] = mass(x);
        s[k] = by_mass ? cbrt(3.0 * x / (4.0 * M_PI * rho_m)) : x;
    }
    return COAG_OK;
}

int coag_create(const coag_grid *g, coag_ctx **out) {
    if (!out) return fail(nullptr, COAG_EINVAL, "coag_create: out is NULL");
    *out = nullptr;
    if (!g || !g->m || !g->m_edge || !g->s)
        return fail(nullptr, COAG_EINVAL, "coag_create: grid or one of its arrays is NULL");
    const int N = g->n_bins;
    if (N < 2 || N > kMaxBins)
        return fail(nullptr, COAG_EINVAL, "coag_create: n_bins = %d outside [2, %d]", N, kMaxBins);
    for (int k = 0; k < N; ++k) {
        if (!(g->m[k] > 0.0) || !(g->s[k] > 0.0))
            return fail(nullptr, COAG_EINVAL, "coag_create: m[%d] or s[%d] not positive", k, k);
        if (k + 1 < N && !(g->m[k + 1] > g->m[k]))
            return fail(nullptr, COAG_EINVAL, "coag_create: m not strictly increasing at %d", k);
        if (!(g->m_edge[k] < g->m[k] && g->m[k] < g->m_edge[k + 1]))
            return fail(nullptr, COAG_EINVAL, "coag_create: m_edge does not bracket m[%d]", k);
    }
    if (!(g->chi > 0.0)) return fail(nullptr, COAG_EINVAL, "coag_create: chi must be > 0");
    if (!(g->eta == g->eta) || g->eta == 2.0)
        return fail(nullptr, COAG_EINVAL, "coag_create: eta must be finite and != 2");
    if (!(g->rho_m > 0.0)) return fail(nullptr, COAG_EINVAL, "coag_create: rho_m must be > 0");
    if (g->split != COAG_SPLIT_MASS && g->split != COAG_SPLIT_NUMBER)
        return fail(nullptr, COAG_EINVAL, "coag_create: unknown split %d", g->split);
    if (g->vertical != 0 && g->vertical != 1)
        return fail(nullptr, COAG_EINVAL, "coag_create: vertical must be 0 or 1, not %d",
                    g->vertical);

    coag_ctx *ctx = new coag_ctx();
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return fail(nullptr, COAG_EHIP, "coag_create: no HIP device");
    }
    if (ctx->device >= 0 && ctx->device < kMaxDevices) {
        // the device address of this device's scratch array, looked up once per
        // device with the device current
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch[ctx->device]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
                (void)hipGetLastError();
                const int dev = ctx->device;
                delete ctx;
                return fail(nullptr, COAG_EHIP,
                            "coag_create: no address for the scratch array on device %d", dev);
            }
            g_scratch[ctx->device] = p;
        }
        ctx->scratch = g_scratch[ctx->device];
    }
    ctx->N = N;
    ctx->P = N * (N + 1) / 2;
    ctx->rho_m = g->rho_m;
    ctx->eta = g->eta;
    ctx->chi = g->chi;
    ctx->split = g->split;
    const size_t P = ctx->P;
    // one block: pij, dst (u32 [P]); cw0, cw1, rw0, rw1, fm ([P]); m, s, dE, invE ([N]);
    // m_edge [N+1]; then the split-precision tables
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    const size_t o_pij = take(4 * P), o_dst = take(4 * P);
    const size_t o_cw0 = take(8 * P), o_cw1 = take(8 * P), o_rw0 = take(8 * P),
                 o_rw1 = take(8 * P), o_fm = take(8 * P);
    const size_t o_m = take(8 * N), o_s = take(8 * N), o_dE = take(8 * N), o_iE = take(8 * N),
                 o_me = take(8 * (N + 1)), o_idm = take(8 * N), o_fc = take(4 * N),
                 o_fr = take(4 * N), o_cd = take(4 * N), o_rd = take(4 * N);
    const size_t o_batch = take(batch_tables_bytes(N));
    if (hipMalloc(&ctx->block, off) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return fail(nullptr, COAG_ENOMEM, "coag_create: table allocation (%zu bytes) failed", off);
    }
    char *b = (char *)ctx->block;
    Tables &T = ctx->T;
    T.N = N;
    T.P = (int)P;
    T.rho_m = g->rho_m;
    T.pij = (uint32_t *)(b + o_pij);
    T.dst = (uint32_t *)(b + o_dst);
    T.cw0 = (double *)(b + o_cw0);
    T.cw1 = (double *)(b + o_cw1);
    T.rw0 = (double *)(b + o_rw0);
    T.rw1 = (double *)(b + o_rw1);
    T.fm = (double *)(b + o_fm);
    T.m = (double *)(b + o_m);
    T.s = (double *)(b + o_s);
    T.dE = (double *)(b + o_dE);
    T.invE = (double *)(b + o_iE);
    T.invdm = (double *)(b + o_idm);
    T.fcol = (int *)(b + o_fc);
    T.frow = (int *)(b + o_fr);
    T.cdiag = (int *)(b + o_cd);
    T.rdiag = (int *)(b + o_rd);
    T.chi = g->chi;
    T.split = g->split;
    T.vertical = g->vertical;
    double *me = (double *)(b + o_me);
    int rc = COAG_OK;
    hipError_t e = hipMemcpy((void *)T.m, g->m, 8 * N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void *)T.s, g->s, 8 * N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(me, g->m_edge, 8 * (N + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_build(N, T.m, me, g->eta, g->chi, g->split, (uint32_t *)T.pij,
                         (uint32_t *)T.dst, (double *)T.cw0, (double *)T.cw1, (double *)T.rw0,
                         (double *)T.rw1, (double *)T.fm, (double *)T.dE, (double *)T.invE,
                         (double *)T.invdm, (int *)T.fcol, (int *)T.frow, (int *)T.cdiag,
                         (int *)T.rdiag, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = build_batch_tables(T, b + o_batch, &ctx->B);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (const char *k = getenv("COAG_STEP_KERNEL")) ctx->batch_fp64 = strcmp(k, "cell") != 0;
    if (const char *k = getenv("COAG_ADJ_SLAB_CELLS")) ctx->adj_slab = atol(k);
    if (e != hipSuccess) rc = fail(nullptr, COAG_EHIP, "coag_create: %s", hipGetErrorString(e));
    if (rc != COAG_OK) {
        (void)hipFree(ctx->block);
        delete ctx;
        return rc;
    }
    *out = ctx;
    return COAG_OK;
}

void coag_destroy(coag_ctx *ctx) {
    if (!ctx) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->block) (void)hipFree(ctx->block);
    if (cur >= 0) (void)hipSetDevice(cur);
    delete ctx;
}

const char *coag_last_error(const coag_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_err.c_str();
}

static int check_cells(coag_ctx *ctx, const coag_cells *c) {
    if (!c || !c->T || !c->rho_g || !c->c_s || !c->Omega || !c->H || !c->nu_mol || !c->alpha)
        return fail(ctx, COAG_EINVAL, "cells or one of its arrays is NULL");
    return COAG_OK;
}

static CellArrays cell_arrays(const coag_cells *c) {
    return CellArrays{c->T, c->rho_g, c->c_s, c->Omega, c->H, c->nu_mol, c->alpha};
}

int coag_rates(coag_ctx *ctx, int64_t C, const coag_cells *cells, const double *v_dust,
               const double *v_frag, double *Kc, double *Kf, void *stream) {
    if (!ctx) return fail(nullptr, COAG_EINVAL, "coag_rates: ctx is NULL");
    if (C < 0 || C > 0x7fffffff) return fail(ctx, COAG_EINVAL, "coag_rates: bad C = %lld", (long long)C);
    if (C == 0) return COAG_OK;                 // nothing to read or write
    if (int r = check_cells(ctx, cells)) return r;
    if (!v_dust || !v_frag || !Kc || !Kf) return fail(ctx, COAG_EINVAL, "coag_rates: NULL array");
    if (int r = set_device(ctx)) return r;
    HIP_TRY(ctx, launch_rates(ctx->T, C, cell_arrays(cells), v_dust, v_frag, Kc, Kf,
                              (hipStream_t)stream));
    return COAG_OK;
}

int coag_rates_blocked(coag_ctx *ctx, int64_t C, const coag_cells *cells, const double *v_dust,
                       const double *v_frag, int32_t f32, void *K, void *stream) {
    if (!ctx) return fail(nullptr, COAG_EINVAL, "coag_rates_blocked: ctx is NULL");
    if (C < 0 || C > 0x7fffffff)
        return fail(ctx, COAG_EINVAL, "coag_rates_blocked: bad C = %lld", (long long)C);
    if (f32 != 0 && f32 != 1) return fail(ctx, COAG_EINVAL, "coag_rates_blocked: f32 must be 0 or 1");
    if (C == 0) return COAG_OK;
    if (int r = check_cells(ctx, cells)) return r;
    if (!v_dust || !v_frag || !K) return fail(ctx, COAG_EINVAL, "coag_rates_blocked: NULL array");
    if (int r = set_device(ctx)) return r;
    HIP_TRY(ctx, launch_rates_blocked(ctx->T, C, cell_arrays(cells), v_dust, v_frag, f32, K,
                                      (hipStream_t)stream));
    return COAG_OK;
}

int coag_rhs(coag_ctx *ctx, int64_t C, const double *rho, const double *Kc, const double *Kf,
             double *drho_dt, void *stream) {
    if (!ctx) return fail(nullptr, COAG_EINVAL, "coag_rhs: ctx is NULL");
    if (C < 0 || C > 0x7fffffff) return fail(ctx, COAG_EINVAL, "coag_rhs: bad C = %lld", (long long)C);
    if (C == 0) return COAG_OK;
    if (!rho || !Kc || !Kf || !drho_dt) return fail(ctx, COAG_EINVAL, "coag_rhs: NULL array");
    if (int r = set_device(ctx)) return r;
    if (reg_path_available(ctx->N))
        HIP_TRY(ctx, launch_rhs2(ctx->T, C, rho, Kc, Kf, drho_dt, (hipStream_t)stream));
    else
        HIP_TRY(ctx, launch_rhs(ctx->T, C, rho, Kc, Kf, drho_dt, (hipStream_t)stream));
    return COAG_OK;
}

// coag_step and coag_step_noalloc: the same checks and kernels; the batched
// step's workspace comes from the context (grown on demand) or, with
// noalloc, from the device's static scratch array (never allocated here)
static int step_impl(const char *fn, coag_ctx *ctx, int64_t C, double *rho, const void *Kc,
                     const void *Kf, double dt, double *h, const coag_tol *tol, int32_t *nsub,
                     int32_t *nrej, double *h_log, int32_t *status, void *stream, bool noalloc) {
    if (!ctx) return fail(nullptr, COAG_EINVAL, "%s: ctx is NULL", fn);
    if (C < 0 || C > 0x7fffffff) return fail(ctx, COAG_EINVAL, "%s: bad C = %lld", fn, (long long)C);
    if (!tol) return fail(ctx, COAG_EINVAL, "%s: tol is NULL", fn);
    const bool blocked = tol->rates_layout != COAG_RATES_CP64;
    if (C > 0 && (!rho || !Kc || (!blocked && !Kf) || !nsub || !status))
        return fail(ctx, COAG_EINVAL, "%s: rho, Kc, Kf ([C][P] rates), nsub and status are "
                    "required", fn);
    if (blocked && Kf)
        return fail(ctx, COAG_EINVAL, "%s: blocked rates hold both kinds in Kc; Kf must be NULL",
                    fn);
    if (!(dt > 0.0) || !isfinite(dt)) return fail(ctx, COAG_EINVAL, "%s: dt must be > 0", fn);
    if (tol->mode < COAG_ADAPTIVE || tol->mode > COAG_REPLAY)
        return fail(ctx, COAG_EINVAL, "%s: unknown mode %d", fn, tol->mode);
    if (tol->prec != COAG_PREC_FP64 && tol->prec != COAG_PREC_SPLIT_BF16)
        return fail(ctx, COAG_EINVAL, "%s: unknown precision %d", fn, tol->prec);
    if (tol->max_sub < 1) return fail(ctx, COAG_EINVAL, "%s: max_sub must be >= 1", fn);
    const int layout = tol->rates_layout;
    if (layout < COAG_RATES_CP64 || layout > COAG_RATES_BLK64)
        return fail(ctx, COAG_EINVAL, "%s: unknown rates_layout %d", fn, layout);
    if (layout == COAG_RATES_BLK32 && tol->prec != COAG_PREC_SPLIT_BF16)
        return fail(ctx, COAG_EINVAL, "%s: FP32 rates need COAG_PREC_SPLIT_BF16", fn);
    if (layout == COAG_RATES_BLK64 && tol->prec != COAG_PREC_FP64)
        return fail(ctx, COAG_EINVAL, "%s: blocked FP64 rates need COAG_PREC_FP64", fn);
    if ((tol->prec == COAG_PREC_SPLIT_BF16 || layout != COAG_RATES_CP64) &&
        !batch_available(ctx->T, ctx->B))
        return fail(ctx, COAG_ENOTSUP,
                    "%s: the split-BF16 step and blocked rates need N >= 16 bins whose "
                    "products of each row fit a 16-bin window, and N <= 343", fn);
    if (layout == COAG_RATES_BLK64 && !ctx->batch_fp64)
        return fail(ctx, COAG_ENOTSUP,
                    "%s: blocked FP64 rates need the batched step "
                    "(COAG_STEP_KERNEL=cell selected the per-cell one)", fn);
    if (tol->mode == COAG_ADAPTIVE) {
        if (!h && C > 0) return fail(ctx, COAG_EINVAL, "%s: h is required in ADAPTIVE mode", fn);
        if (!(tol->rtol > 0.0) || !(tol->atol_rel >= 0.0) || !(tol->h_min_rel >= 0.0))
            return fail(ctx, COAG_EINVAL, "%s: need rtol > 0, atol_rel >= 0, h_min_rel >= 0", fn);
    }
    if (tol->mode == COAG_REPLAY && !h_log && C > 0)
        return fail(ctx, COAG_EINVAL, "%s: h_log is required in REPLAY mode", fn);
    if (C == 0) return COAG_OK;
    if (int r = set_device(ctx)) return r;
    StepArgs a;
    a.rho = rho;
    a.Kc = (const double *)Kc;
    a.Kf = (const double *)Kf;
    a.dt = dt;
    a.h = h;
    a.rtol = tol->rtol;
    a.atol_rel = tol->atol_rel;
    a.h_min_rel = tol->h_min_rel;
    a.max_sub = tol->max_sub;
    a.mode = tol->mode;
    a.renorm = tol->renorm;
    a.nsub = nsub;
    a.nrej = nrej;
    a.status = status;
    a.h_log = h_log;
    const bool split = tol->prec == COAG_PREC_SPLIT_BF16;
    if (split || (ctx->batch_fp64 && batch_available(ctx->T, ctx->B))) {
        const size_t need = batch_ws_bytes(ctx->N, C, split ? 1 : 0, layout);
        double *ws;
        if (noalloc) {
            if (!ctx->scratch)
                return fail(ctx, COAG_ENOTSUP, "%s: no scratch array on device %d", fn,
                            ctx->device);
            if (need > kScratchBytes)
                return fail(ctx, COAG_EINVAL,
                            "%s: %lld cells of %d bins need %zu bytes of scratch, more than its "
                            "%zu bytes; split the call into fewer cells", fn, (long long)C,
                            ctx->N, need, kScratchBytes);
            ws = (double *)ctx->scratch;
        } else {
            if (int r = ensure_ws(ctx, need)) return r;
            ws = (double *)ctx->ws;
        }
        HIP_TRY(ctx, launch_step_batch(ctx->T, ctx->B, C, a, split ? 1 : 0, layout, ws,
                                       (hipStream_t)stream));
    } else if (reg_path_available(ctx->N)) {
        HIP_TRY(ctx, launch_step2(ctx->T, C, a, (hipStream_t)stream));
    } else {
        HIP_TRY(ctx, launch_step(ctx->T, C, a, (hipStream_t)stream));
    }
    return COAG_OK;
}

int coag_step(coag_ctx *ctx, int64_t C, double *rho, const void *Kc, const void *Kf,
              double dt, double *h, const coag_tol *tol, int32_t *nsub, int32_t *nrej,
              double *h_log, int32_t *status, void *stream) {
    return step_impl("coag_step", ctx, C, rho, Kc, Kf, dt, h, tol, nsub, nrej, h_log, status,
                     stream, false);
}

int coag_step_noalloc(coag_ctx *ctx, int64_t C, double *rho, const void *Kc, const void *Kf,
                      double dt, double *h, const coag_tol *tol, int32_t *nsub, int32_t *nrej,
                      double *h_log, int32_t *status, void *stream) {
    return step_impl("coag_step_noalloc", ctx, C, rho, Kc, Kf, dt, h, tol, nsub, nrej, h_log,
                     status, stream, true);
}

// Workspace of the batched adjoint per slab of S cells (S a multiple of 16,
// or all C cells): blocked rates (RT) and rate derivatives (GT), the forward
// replay's step starts Ys and stage states Zs, the replay's state, slopes and
// status, and v3.  (Zf, Xf: the rate-derivative factors Z, X.)
struct AdjWs {
    size_t K, Zf, Xf, Wf, Ys, Zs, y, slopes, status, v3, total;
};

static AdjWs adj_ws(int N, size_t P, long S, int L, int split, int gf32, bool vertical) {
    const size_t Sb = ((size_t)S + kBatchCells - 1) / kBatchCells * kBatchCells;
    const size_t rt = split ? 4 : 8, gt = gf32 ? 4 : 8;
    AdjWs w;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += align256(b); return r; };
    w.K = take(rt * 64 * (size_t)pair_slot0(N) * (Sb / kBatchCells));   // blocked, both kinds
    w.Zf = take(gt * P * Sb);
    w.Xf = take(gt * P * Sb);
    w.Wf = vertical ? take(gt * P * Sb) : 0;
    w.Ys = take(8 * (size_t)N * (size_t)(L + 1) * (size_t)S);
    w.Zs = take(8 * (size_t)N * 2 * (size_t)L * (size_t)S);
    w.y = take(8 * (size_t)N * (size_t)S);
    w.slopes = take(batch_ws_bytes(N, S, split, split ? COAG_RATES_BLK32 : COAG_RATES_BLK64));
    w.status = take(4 * (size_t)S);
    w.v3 = take(8 * (size_t)N * (size_t)S);
    w.total = o;
    return w;
}

// cells per slab: all of them if their workspace fits the budget, else the
// fewest slabs of whole 16-cell batches that fit it (at least 4096 cells, a
// launch that still fills the GPU), all of about the same size
constexpr size_t kAdjBudget = (size_t)8 << 30;

static long adj_slab_cells(const coag_ctx *ctx, long C, int L, int split, int gf32) {
    if (ctx->adj_slab > 0) {
        const long s = (ctx->adj_slab + kBatchCells - 1) / kBatchCells * kBatchCells;
        return s < C ? s : C;
    }
    const bool vt = ctx->T.vertical != 0;
    if (adj_ws(ctx->N, ctx->P, C, L, split, gf32, vt).total <= kAdjBudget) return C;
    const size_t per16 = adj_ws(ctx->N, ctx->P, 16, L, split, gf32, vt).total;
    long smax = (long)(kAdjBudget / per16) * kBatchCells;
    if (smax < 4096) smax = 4096;
    const long nslab = (C + smax - 1) / smax;
    const long s = ((C + nslab - 1) / nslab + kBatchCells - 1) / kBatchCells * kBatchCells;
    return s < C ? s : C;
}

int coag_step_backward(coag_ctx *ctx, int64_t C, const double *rho_in, const coag_cells *cells,
                       const double *v_dust, const double *v_frag, const double *h_log,
                       int32_t log_stride, const int32_t *nsub, const double *g_out,
                       double *g_in, double *g_alpha, double *g_vfrag, int32_t prec,
                       void *stream) {
    if (!ctx) return fail(nullptr, COAG_EINVAL, "coag_step_backward: ctx is NULL");
    if (C < 0 || C > 0x7fffffff)
        return fail(ctx, COAG_EINVAL, "coag_step_backward: bad C = %lld", (long long)C);
    if (prec != COAG_PREC_FP64 && prec != COAG_PREC_SPLIT_BF16)
        return fail(ctx, COAG_EINVAL, "coag_step_backward: unknown precision %d", prec);
    if (log_stride < 1) return fail(ctx, COAG_EINVAL, "coag_step_backward: log_stride must be >= 1");
    const bool split = prec == COAG_PREC_SPLIT_BF16;
    const bool batched = adj_batch_available(ctx->T, ctx->B) && (split || ctx->batch_fp64);
    if (split && !batched)
        return fail(ctx, COAG_ENOTSUP,
                    "coag_step_backward: the split-BF16 adjoint needs the batched kernels "
                    "(N >= 16 bins whose products of each row fit a 16-bin window, and the "
                    "state of 16 cells within the LDS of one workgroup)");
    if (ctx->T.vertical && !batched)
        return fail(ctx, COAG_ENOTSUP,
                    "coag_step_backward: the adjoint of the vertically integrated kernel "
                    "needs the batched kernels (the per-cell adjoint has the volume kernel's "
                    "rate derivatives only)");
    if (C == 0) return COAG_OK;
    if (int r = check_cells(ctx, cells)) return r;
    if (!rho_in || !v_dust || !v_frag || !h_log || !nsub || !g_out || !g_in || !g_alpha || !g_vfrag)
        return fail(ctx, COAG_EINVAL, "coag_step_backward: NULL array");
    if (int r = set_device(ctx)) return r;
    const size_t P = ctx->P, N = ctx->N;
    const CellArrays ca = cell_arrays(cells);
    hipStream_t st = (hipStream_t)stream;
    if (batched) {
        // per slab: rates and their derivatives (blocked), the forward replay
        // keeping every step's start and stage states, then the reverse sweep
        const int gf32 = split ? 1 : 0;
        const int L = log_stride;
        const long S = adj_slab_cells(ctx, C, L, split, gf32);
        const AdjWs w = adj_ws(ctx->N, P, S, L, split, gf32, ctx->T.vertical != 0);
        if (int r = ensure_ws(ctx, w.total)) return r;
        char *b = (char *)ctx->ws;
        for (long s0 = 0; s0 < C; s0 += S) {
            const long Cs = C - s0 < S ? C - s0 : S;
            const CellArrays cs{ca.T + s0, ca.rho_g + s0, ca.c_s + s0, ca.Omega + s0,
                                ca.H + s0, ca.nu_mol + s0, ca.alpha + s0};
            const double *vd = v_dust + (size_t)s0 * N * 3, *vf = v_frag + s0;
            HIP_TRY(ctx, launch_rates_blocked(ctx->T, Cs, cs, vd, vf, split ? 1 : 0, b + w.K, st));
            HIP_TRY(ctx, launch_rate_derivs_blocked(ctx->T, Cs, cs, vd, vf, gf32, b + w.Zf,
                                                    b + w.Xf, ctx->T.vertical ? b + w.Wf : nullptr,
                                                    st));
            double *y = (double *)(b + w.y);
            HIP_TRY(ctx, hipMemcpyAsync(y, rho_in + (size_t)s0 * N, 8 * N * (size_t)Cs,
                                        hipMemcpyDeviceToDevice, st));
            StepArgs sa;
            sa.rho = y;
            sa.Kc = (const double *)(b + w.K);
            sa.Kf = nullptr;
            sa.dt = 0.0;
            sa.h = nullptr;
            sa.rtol = sa.atol_rel = sa.h_min_rel = 0.0;
            sa.max_sub = L;
            sa.mode = COAG_REPLAY;
            sa.renorm = 0;
            sa.nsub = const_cast<int32_t *>(nsub + s0);            // read only in REPLAY
            sa.nrej = nullptr;
            sa.status = (int32_t *)(b + w.status);
            sa.h_log = const_cast<double *>(h_log + (size_t)s0 * L);  // read only in REPLAY
            sa.Ys = (double *)(b + w.Ys);
            sa.Zs = (double *)(b + w.Zs);
            HIP_TRY(ctx, launch_step_batch(ctx->T, ctx->B, Cs, sa, split ? 1 : 0,
                                           split ? COAG_RATES_BLK32 : COAG_RATES_BLK64,
                                           (double *)(b + w.slopes), st));
            AdjBatchArgs aa;
            aa.Kc = b + w.K;
            aa.Kf = nullptr;
            aa.Z = b + w.Zf;
            aa.X = b + w.Xf;
            aa.W = ctx->T.vertical ? b + w.Wf : nullptr;
            aa.v_frag = vf;
            aa.Ys = sa.Ys;
            aa.Zs = sa.Zs;
            aa.h_log = h_log + (size_t)s0 * L;
            aa.L = L;
            aa.nsub = nsub + s0;
            aa.status = sa.status;
            aa.g_out = g_out + (size_t)s0 * N;
            aa.g_in = g_in + (size_t)s0 * N;
            aa.v3 = (double *)(b + w.v3);
            aa.g_alpha = g_alpha + s0;
            aa.g_vfrag = g_vfrag + s0;
            HIP_TRY(ctx, launch_adjoint_batch(ctx->T, ctx->B, Cs, aa, split ? 1 : 0, gf32, st));
        }
        return COAG_OK;
    }
    // one cell per workgroup (grids the batched kernels do not cover, or
    // COAG_STEP_KERNEL=cell): rates [C][P], dJ/dK per pair, stage states
    const size_t bK = align256(8 * P * (size_t)C);
    const size_t bY = align256(8 * N * (size_t)(log_stride + 1) * (size_t)C);
    const size_t bZ = align256(8 * N * 2 * (size_t)log_stride * (size_t)C);
    if (int r = ensure_ws(ctx, 4 * bK + bY + bZ)) return r;
    char *w = (char *)ctx->ws;
    double *Kc = (double *)w, *Kf = (double *)(w + bK), *gKc = (double *)(w + 2 * bK),
           *gKf = (double *)(w + 3 * bK), *Ys = (double *)(w + 4 * bK);
    double *Zs = (double *)(w + 4 * bK + bY);
    HIP_TRY(ctx, launch_rates(ctx->T, C, ca, v_dust, v_frag, Kc, Kf, st));
    AdjArgs a;
    a.rho_in = rho_in;
    a.Kc = Kc;
    a.Kf = Kf;
    a.gKc = gKc;
    a.gKf = gKf;
    a.Ys = Ys;
    a.Zs = Zs;
    a.replayed = 0;
    a.h_log = h_log;
    a.log_stride = log_stride;
    a.nsub = nsub;
    a.g_out = g_out;
    a.g_in = g_in;
    HIP_TRY(ctx, launch_adjoint(ctx->T, C, a, ca, v_dust, v_frag, g_alpha, g_vfrag, st));
    return COAG_OK;
}

}  // extern "C"
