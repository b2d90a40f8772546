// coag_split.h -- split-BF16 MFMA contraction of the gain/loss terms.
#pragma once

#include <hip/hip_runtime.h>

#include "coag_launch.h"

namespace coag {

struct SplitTables {
    int available;
};

size_t split_tables_bytes(int N);
hipError_t build_split_tables(const Tables &T, void *mem, SplitTables *S, hipStream_t st);
size_t split_step_ws_bytes(int N, long C);
hipError_t launch_step_split(const Tables &T, const SplitTables &S, long C, const StepArgs &a,
                             void *ws, hipStream_t st);
size_t split_adjoint_ws_bytes(int N, long C);
hipError_t launch_adjoint_split(const Tables &T, const SplitTables &S, long C, const AdjArgs &a,
                                const CellArrays &cells, const double *v_dust,
                                const double *v_frag, double *g_alpha, double *g_vfrag, void *ws,
                                hipStream_t st);

}  // namespace coag
