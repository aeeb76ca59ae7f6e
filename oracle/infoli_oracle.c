/*
 * Plain CPU oracle of the InfOli simulation step (arXiv:1612.01501).
 *
 * TEST INFRASTRUCTURE ONLY. This file checks the GPU library; it is not part
 * of it. Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it. It shares no code, header, table or helper with the
 * HIP library, and includes nothing from it.
 *
 * What it computes (Section 2.2 and Section 2.3.1 of the paper):
 *   - every step n -> n+1 updates all three compartments of every cell and
 *     all gap junctions from the step-n state only (synchronous, "Jacobi"
 *     forward Euler with dt = 50 us);
 *   - the gap current into cell i is sum_j w_ij*dV*(0.8*exp(-dV^2/100)+0.2),
 *     dV = Vd_i - Vd_j (Algorithm 1, odd form, see orc_gap);
 *   - the evoked input is one value per neuron per step (Table 1).
 * The cell equations are not printed in the paper; they follow the published
 * three-compartment model it cites (see orc_rhs). Their constants appear in
 * this file only.
 *
 * Built twice from oracle_body.inc: *_f64 (double) and *_f32 (float, every
 * operation in float, libm expf/expm1f, IEEE division, no fast-math).
 *
 * Parity pins: see tests/test_oracle_pins.py. Absolute trajectories against
 * the paper are parity unpinned (the paper prints no trajectory values).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* connectivity kinds */
#define ORC_CONN_NONE 0
#define ORC_CONN_UNIFORM_ALL 1
#define ORC_CONN_DENSE 2
#define ORC_CONN_CSR 3

/* state variables, structure-of-arrays order */
#define ORC_S_VD 0  /* dendrite voltage (mV)                          */
#define ORC_S_CA 1  /* dendritic [Ca2+]                               */
#define ORC_S_R 2   /* high-threshold Ca activation                   */
#define ORC_S_S 3   /* Ca-activated K activation                      */
#define ORC_S_Q 4   /* h-current activation                           */
#define ORC_S_VS 5  /* soma voltage (mV)                              */
#define ORC_S_K 6   /* low-threshold Ca activation                    */
#define ORC_S_L 7   /* low-threshold Ca inactivation                  */
#define ORC_S_H 8   /* soma Na inactivation                           */
#define ORC_S_N 9   /* soma delayed-rectifier K activation            */
#define ORC_S_X 10  /* soma K activation (alpha/beta form)            */
#define ORC_S_VA 11 /* axon voltage (mV), the cell output             */
#define ORC_S_HA 12 /* axon Na inactivation                           */
#define ORC_S_XA 13 /* axon K activation                              */
#define ORC_S 14

/* the 20 per-cell conductances / reversal potentials (Table 1: 20 values) */
#define ORC_P_G_CAH 0
#define ORC_P_G_KCA 1
#define ORC_P_G_H 2
#define ORC_P_G_LD 3
#define ORC_P_G_CAL 4
#define ORC_P_G_NA_S 5
#define ORC_P_G_KDR_S 6
#define ORC_P_G_K_S 7
#define ORC_P_G_LS 8
#define ORC_P_G_NA_A 9
#define ORC_P_G_K_A 10
#define ORC_P_G_LA 11
#define ORC_P_G_INT 12
#define ORC_P_P1 13
#define ORC_P_P2 14
#define ORC_P_V_NA 15
#define ORC_P_V_K 16
#define ORC_P_V_CA 17
#define ORC_P_V_H 18
#define ORC_P_V_L 19
#define ORC_P 20

int orc_num_state_vars(void) { return ORC_S; }
int orc_num_params(void) { return ORC_P; }
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define REAL double
#define SFX(name) name##_f64
#define EXP exp
#define EXPM1 expm1
#include "oracle_body.inc"
#undef REAL
#undef SFX
#undef EXP
#undef EXPM1

#define REAL float
#define SFX(name) name##_f32
#define EXP expf
#define EXPM1 expm1f
#include "oracle_body.inc"
#undef REAL
#undef SFX
#undef EXP
#undef EXPM1
