// coag_batch.h -- the cell-batched step (coag_batch.hip): 16 cells per
// workgroup advance in lockstep and the gain contraction of every right-hand
// side runs on the matrix cores, in FP64 or as split-BF16 products.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "coag_launch.h"

namespace coag {

// Chunk tables of the batched contraction, built once per context.
//   chunk = (row i, column block q): the pairs (i, j), j in [16q, 16q + 16),
//   j <= i; NC chunks, listed row by row (crow, FP64 form) and column block by
//   column block (crow_c, split form).  Every product of row i (coagulation
//   and remnant targets, and bin i itself, which loses m_i per collision) lies
//   in the 16-bin window [wb[i], wb[i] + 16).
//   b64: FP64 B operands of v_mfma_f64_16x16x4f64 in crow order, [NC][4][64][2]
//        (operand s of lane l at [s / 2][l][s % 2]: a lane's pairs of operands
//        are 16-byte loads, contiguous over the wave)
//   b16: three BF16 limbs of the same entries for v_mfma_f32_16x16x32_bf16, in
//        crow_c order, [NC][3][64] x 16 bytes
//   a64: the same entries as A operands of the adjoint's v_mfma_f64_16x16x4f64
//        (pairs as rows, bins as the K dimension), crow_c order, operand
//        e = 4 kind + t of lane l at [NC][e / 2][64][e % 2] (16-byte loads):
//        lane l holds pair 16q + l % 16, bin wb[i] + 4 t + l / 16
//   a16: three BF16 limbs of the adjoint's A operands of
//        v_mfma_f32_16x16x32_bf16, crow_c order, [NC][2 kinds][3 limbs][32] x
//        16 bytes: entry l holds pair 16q + l % 16, bins wb[i] + 8 (l / 16) + e,
//        e = 0..7
struct BatchTables {
    int NC;
    int ok;                      // every row fits its window (else the path is off)
    const int *crow;             // [NC]  i | q << 16, row by row
    const int *crow_c;           // [NC]  i | q << 16, column block by column block
    const int *wb;               // [N]
    const double *b64;
    const uint4 *b16;
    const double *a64;
    const uint4 *a16;
};

constexpr int kBatchCells = 16;

size_t batch_tables_bytes(int N);
// builds the tables into `mem`; reads back (synchronously) whether every row
// fits its window
hipError_t build_batch_tables(const Tables &T, void *mem, BatchTables *B);
// whether the batched step runs for this context (window fit, LDS size)
bool batch_available(const Tables &T, const BatchTables &B);
// workspace of a batched step: four slopes and the candidate state per cell,
// and (FP64 form from [C][P] rates) the rates of every batch reordered
// pair-major with the cells innermost
size_t batch_ws_bytes(int N, long C, int prec, int layout);
// prec: 0 = FP64 MFMA, 1 = split BF16.  layout of Kc / Kf: 0 = double [C][P],
// 1 = float 16-cell-blocked (split only), 2 = double 16-cell-blocked (FP64
// only); hipErrorNotSupported for other combinations
// ws: batch_ws_bytes(N, C, prec, layout) bytes, or, with wk given, the
// slope part only and wk the [C][P] reordering area (FP64 [C][P] rates)
// Reverse sweep of the batched adjoint (coag_adjoint.hip) over a frozen step
// sequence, for C cells whose rates (blocked, RT = float or double) and
// rate-derivative factors Z, X (blocked, GT; pair_rate_derivs) are given; Ys,
// Zs hold the forward replay's step starts and stage states (layout of
// AdjArgs, stride L = log_stride).
struct AdjBatchArgs {
    const void *Kc, *Kf;                 // Kc: the blocked rates (blk_elem), RT; Kf unused
    const void *Z, *X;                   // [ceil(C/16)][P][16] GT
    const void *W;                       // the same, vertically integrated kernel only
    const double *v_frag;                // [C]
    const double *Ys, *Zs;
    const double *h_log;
    int L;
    const int32_t *nsub;
    const int32_t *status;               // replay status per cell (non-zero: outputs NaN)
    const double *g_out;
    double *g_in;                        // may equal g_out
    double *v3;                          // workspace [C][N]
    double *g_alpha, *g_vfrag;
};

// whether the batched adjoint runs for this context (the batched step does,
// and its LDS fits)
bool adj_batch_available(const Tables &T, const BatchTables &B);
// the rate-derivative factors Z, X (pair_rate_derivs), and W of the
// vertically integrated kernel (T.vertical; W unused otherwise), in the
// 16-cell-blocked layout, double (f32 = 0) or float (f32 = 1)
hipError_t launch_rate_derivs_blocked(const Tables &T, long C, const CellArrays &cells,
                                      const double *v_dust, const double *v_frag, int f32,
                                      void *Z, void *X, void *W, hipStream_t st);
// prec 0: FP64 rates and derivatives, FP64 matrix cores; prec 1: FP32 rates,
// derivatives of type given by gf32, split-BF16 matrix products
hipError_t launch_adjoint_batch(const Tables &T, const BatchTables &B, long C,
                                const AdjBatchArgs &a, int prec, int gf32, hipStream_t st);

hipError_t launch_step_batch(const Tables &T, const BatchTables &B, long C, const StepArgs &a,
                             int prec, int layout, double *ws, hipStream_t st,
                             void *wk = nullptr);

}  // namespace coag
