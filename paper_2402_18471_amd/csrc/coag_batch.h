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
//   b64: FP64 B operands of v_mfma_f64_16x16x4f64 in crow order, [NC][8][64]
//   b16: three BF16 limbs of the same entries for v_mfma_f32_16x16x32_bf16, in
//        crow_c order, [NC][3][64] x 16 bytes
struct BatchTables {
    int NC;
    int ok;                      // every row fits its window (else the path is off)
    const int *crow;             // [NC]  i | q << 16, row by row
    const int *crow_c;           // [NC]  i | q << 16, column block by column block
    const int *wb;               // [N]
    const double *b64;
    const uint4 *b16;
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
hipError_t launch_step_batch(const Tables &T, const BatchTables &B, long C, const StepArgs &a,
                             int prec, int layout, double *ws, hipStream_t st,
                             void *wk = nullptr);

}  // namespace coag
