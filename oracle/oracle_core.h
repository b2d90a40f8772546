/*
 * oracle_core.h -- internal declarations of the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: the oracle is a plain, slow FP64 reference for the
 * coagulation-fragmentation update of Robinson, Booth & Owen (cuDisc), Sec. 5.
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or constant generator with the GPU
 * library.
 */
#ifndef ORACLE_CORE_H
#define ORACLE_CORE_H

#include <stdint.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORACLE_KB 1.380649e-16        /* Boltzmann constant, erg/K (CGS) */
#define ORACLE_YSTAR 1.6              /* St* / St_1 in the intermediate regime */
#define ORACLE_PSERIES_Y 1.0e-2       /* below this y, p_coag uses its series */

enum { ORACLE_SPLIT_MASS = 0, ORACLE_SPLIT_NUMBER = 1 };
enum { ORACLE_ADAPTIVE = 0, ORACLE_FIXED = 1, ORACLE_REPLAY = 2 };
enum { ORACLE_CELL_OK = 0, ORACLE_CELL_HMIN = 1, ORACLE_CELL_MAXSUB = 2,
       ORACLE_CELL_NONFINITE = 3 };

/* Mass grid and collision-outcome parameters, as handed in by the caller. */
typedef struct {
    int32_t N;
    int32_t split;                    /* ORACLE_SPLIT_* */
    const double *m, *m_edge, *s;     /* [N], [N+1], [N] */
    double rho_m, eta, chi;
    int32_t vertical;                 /* 1: vertically integrated kernel (Sec. 5.1) */
} oracle_grid_t;

/* Per-cell gas state, one value per cell for each array. */
typedef struct {
    const double *T, *rho_g, *c_s, *Omega, *H, *nu_mol, *alpha;
} oracle_cells_t;

typedef struct {
    double rtol, atol_rel, h_min_rel;
    int32_t max_sub, mode;
} oracle_tol_t;

/* Where each pair's collision products go (Sec. 5, eqs. `Cijk`, `Rijk`,
   `Nijk`, `fragrem`).  Indexed by packed pair p = i(i+1)/2 + j, j <= i. */
typedef struct {
    int N;
    long P;
    const double *m, *m_edge, *s;
    double rho_m;
    int vertical;                     /* vertically integrated kernel */
    int *ci;  double *cw0, *cw1;      /* coagulation: lower bin, mass into ci, ci+1 */
    int *ri;  double *rw0, *rw1;      /* remnant:     lower bin, mass into ri, ri+1 */
    int *fl;  double *fm;             /* fragments:   top bin l, total fragment mass */
    double *Nfrac;                    /* [N][N]: Nfrac[l][k] = N_k(m^e_{l+1}), k <= l */
    int *pi, *pj;                     /* pair -> (i, j) */
} ored;

int  ored_build(const oracle_grid_t *g, ored *r);
void ored_free(ored *r);

#endif
