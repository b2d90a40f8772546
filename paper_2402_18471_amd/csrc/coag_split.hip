// coag_split.hip -- split-BF16 MFMA form of the contraction (not yet built).
#include "coag_split.h"

namespace coag {

size_t split_tables_bytes(int) { return 256; }
hipError_t build_split_tables(const Tables &, void *, SplitTables *S, hipStream_t) {
    S->available = 0;
    return hipSuccess;
}
size_t split_step_ws_bytes(int, long) { return 0; }
hipError_t launch_step_split(const Tables &, const SplitTables &, long, const StepArgs &, void *,
                             hipStream_t) {
    return hipErrorNotSupported;
}
size_t split_adjoint_ws_bytes(int, long) { return 0; }
hipError_t launch_adjoint_split(const Tables &, const SplitTables &, long, const AdjArgs &,
                                const CellArrays &, const double *, const double *, double *,
                                double *, void *, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace coag
