// coag_launch.h -- argument blocks and launchers shared by the host API
// (coag_api.hip) and the kernels (coag_kernels.hip, coag_step2.hip, coag_batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "coag_device.h"

namespace coag {

struct CellArrays {
    const double *T, *rho_g, *c_s, *Omega, *H, *nu_mol, *alpha;
};

struct StepArgs {
    double *rho;
    const double *Kc, *Kf;
    double dt;
    double *h;
    double rtol, atol_rel, h_min_rel;
    int max_sub, mode, renorm;
    int32_t *nsub, *nrej, *status;
    double *h_log;
    // REPLAY on the batched step only: where to keep the step-start states
    // and the inner stage states y2, y3 of every sub-step, laid out as
    // AdjArgs::Ys and AdjArgs::Zs with log_stride = max_sub; nullptr: not kept
    double *Ys = nullptr, *Zs = nullptr;
};

struct AdjArgs {
    const double *rho_in;
    const double *Kc, *Kf;       // rates of the cells (workspace)
    double *gKc, *gKf;           // dJ/dKc, dJ/dKf (workspace)
    double *Ys;                  // step-start states (workspace) [C][log_stride+1][N]
    double *Zs;                  // inner stage states y2, y3 (workspace) [C][log_stride][2][N]
    const double *h_log;
    int log_stride;
    const int32_t *nsub;
    const double *g_out;
    double *g_in;
    int replayed = 0;            // Ys, Zs already hold the forward replay
};

hipError_t launch_build(int N, const double *m, const double *me, double eta, double chi,
                        int split, uint32_t *pij, uint32_t *dst, double *cw0, double *cw1,
                        double *rw0, double *rw1, double *fm, double *dE, double *invE,
                        double *invdm, int *fcol, int *frow, int *cdiag, int *rdiag,
                        hipStream_t st);
hipError_t launch_rates(const Tables &T, long C, const CellArrays &cells, const double *v_dust,
                        const double *v_frag, double *Kc, double *Kf, hipStream_t st);
// rates in the 16-cell-blocked layout (blk_elem: both kinds in one array),
// float (f32) or double
hipError_t launch_rates_blocked(const Tables &T, long C, const CellArrays &cells,
                                const double *v_dust, const double *v_frag, int f32, void *K,
                                hipStream_t st);
hipError_t launch_rhs(const Tables &T, long C, const double *rho, const double *Kc,
                      const double *Kf, double *out, hipStream_t st);
size_t step_lds_bytes(int N);
hipError_t launch_step(const Tables &T, long C, const StepArgs &a, hipStream_t st);
// register-resident FP64 path (coag_step2.hip), for bin counts whose pair
// triangle fits the registers of one workgroup
bool reg_path_available(int N);
hipError_t launch_rhs2(const Tables &T, long C, const double *rho, const double *Kc,
                       const double *Kf, double *out, hipStream_t st);
hipError_t launch_step2(const Tables &T, long C, const StepArgs &a, hipStream_t st);
hipError_t launch_adjoint(const Tables &T, long C, const AdjArgs &a, const CellArrays &cells,
                          const double *v_dust, const double *v_frag, double *g_alpha,
                          double *g_vfrag, hipStream_t st);

}  // namespace coag
