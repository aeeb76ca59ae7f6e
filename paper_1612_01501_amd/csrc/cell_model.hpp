// Device-side InfOli cell: one forward-Euler step of the three-compartment
// inferior-olive neuron (dendrite, soma, axon) from its previous-step state.
//
// The paper (Section 2.2) treats the cell model as given: 3 compartments,
// one evoked input into the dendrite, the axon voltage as output, every
// quantity of step n+1 computed from step n. The equations restate the
// published model it cites (De Gruijl et al., PLoS Comput Biol 8, 2012,
// built on Schweighofer et al., J Neurophysiol 82, 1999): Hodgkin-Huxley
// currents with sigmoid or alpha/beta gates, a first-order dendritic
// calcium pool, and ohmic coupling between compartments scaled by the
// soma/dendrite (p1) and axon/soma (p2) area ratios.
#pragma once
#include <hip/hip_runtime.h>

namespace infoli {

enum : int {
    SV_VD = 0, SV_CA, SV_R, SV_S, SV_Q, SV_VS, SV_K, SV_L, SV_H, SV_N, SV_X,
    SV_VA, SV_HA, SV_XA, NSV
};

// The 20 per-cell values (conductances mS/cm^2, area ratios, reversal mV).
struct CellParams {
    float gCaH, gKCa, gH, gLd, gCaL, gNaS, gKdrS, gKS, gLs, gNaA, gKA, gLa;
    float gInt, p1, p2;
    float eNa, eK, eCa, eH, eL;
};
static_assert(sizeof(CellParams) == 20 * sizeof(float), "20 parameters");

// x / (exp(x/s) - 1), continuous at x = 0 where it equals s.
__device__ __forceinline__ float ratio_expm1(float x, float s) {
    return (x == 0.0f) ? s : x / expm1f(x / s);
}

// Steady-state curve 1/(1 + exp(-(v - vh)/k)); k < 0 for inactivation.
__device__ __forceinline__ float boltz(float v, float vh, float k) {
    return 1.0f / (1.0f + expf(-(v - vh) / k));
}

// The update is Jacobi (every derivative from the previous-step state), so
// each compartment's next state is a function of x alone; the three parts
// below write disjoint entries of y and together are cell_step.

// Dendrite part: y[Vd, Ca, r, s, q]. igap: gap current leaving the dendrite,
// iapp: evoked input into the dendrite, dt in ms.
__device__ __forceinline__ void cell_step_dendrite(const CellParams& p, const float* __restrict__ x,
                                                   float igap, float iapp, float dt, float* __restrict__ y) {
    const float vd = x[SV_VD], vs = x[SV_VS];

    // Dendrite: high-threshold Ca (r^2), Ca-activated K (s), h current (q),
    // leak, coupling to the soma, gap junctions and the evoked input.
    const float icah = p.gCaH * x[SV_R] * x[SV_R] * (vd - p.eCa);
    const float ikca = p.gKCa * x[SV_S] * (vd - p.eK);
    const float ih = p.gH * x[SV_Q] * (vd - p.eH);
    const float ild = p.gLd * (vd - p.eL);
    const float ids = p.gInt / (1.0f - p.p1) * (vd - vs);
    const float dvd = iapp - igap - ids - icah - ikca - ih - ild;

    const float dca = -3.0f * icah - 0.075f * x[SV_CA];

    const float ar = 1.7f / (1.0f + expf(-(vd - 5.0f) / 13.9f));
    const float br = 0.02f * ratio_expm1(vd + 8.5f, 5.0f);
    const float dr = (ar - (ar + br) * x[SV_R]) / 5.0f;

    const float as = fminf(0.00002f * x[SV_CA], 0.01f);
    const float ds = as - (as + 0.015f) * x[SV_S];

    const float qinf = boltz(vd, -80.0f, -4.0f);
    const float rq = expf(-0.086f * vd - 14.6f) + expf(0.070f * vd - 1.87f);  // 1/tau_q
    const float dq = (qinf - x[SV_Q]) * rq;

    // C_m = 1 uF/cm^2: dV/dt equals the net inward current density.
    y[SV_VD] = vd + dt * dvd;
    y[SV_CA] = x[SV_CA] + dt * dca;
    y[SV_R] = x[SV_R] + dt * dr;
    y[SV_S] = x[SV_S] + dt * ds;
    y[SV_Q] = x[SV_Q] + dt * dq;
}

// Soma part: y[Vs, k, l, h, n, x].
__device__ __forceinline__ void cell_step_soma(const CellParams& p, const float* __restrict__ x, float dt,
                                               float* __restrict__ y) {
    const float vd = x[SV_VD], vs = x[SV_VS], va = x[SV_VA];

    // Soma: low-threshold Ca (k^3 l), Na (instantaneous m^3, h), delayed
    // rectifier K (n^4), K (x^4), leak, coupling to dendrite and axon.
    const float kk = x[SV_K];
    const float icaL = p.gCaL * kk * kk * kk * x[SV_L] * (vs - p.eCa);
    const float ms = boltz(vs, -30.0f, 5.5f);
    const float inas = p.gNaS * ms * ms * ms * x[SV_H] * (vs - p.eNa);
    const float n2 = x[SV_N] * x[SV_N];
    const float ikdr = p.gKdrS * n2 * n2 * (vs - p.eK);
    const float x2 = x[SV_X] * x[SV_X];
    const float iks = p.gKS * x2 * x2 * (vs - p.eK);
    const float ils = p.gLs * (vs - p.eL);
    const float isd = p.gInt / p.p1 * (vs - vd);
    const float isa = p.gInt / (1.0f - p.p2) * (vs - va);
    const float dvs = -(icaL + inas + ikdr + iks + ils + isd + isa);

    const float dk = boltz(vs, -61.0f, 4.2f) - kk;                  // tau_k = 1 ms
    const float taul = 20.0f * expf((vs + 160.0f) / 30.0f) / (1.0f + expf((vs + 84.0f) / 7.3f)) + 35.0f;
    const float dl = (boltz(vs, -85.5f, -8.5f) - x[SV_L]) / taul;
    const float tauh = 3.0f * expf(-(vs + 40.0f) / 33.0f);
    const float dh = (boltz(vs, -70.0f, -5.8f) - x[SV_H]) / tauh;
    const float taun = 5.0f + 47.0f * expf((vs + 50.0f) / 900.0f);
    const float dn = (boltz(vs, -3.0f, 10.0f) - x[SV_N]) / taun;
    const float axs = 0.13f * ratio_expm1(-(vs + 25.0f), 10.0f);
    const float bxs = 1.69f * expf(-0.0125f * (vs + 35.0f));
    const float dx = axs - (axs + bxs) * x[SV_X];

    y[SV_VS] = vs + dt * dvs;
    y[SV_K] = kk + dt * dk;
    y[SV_L] = x[SV_L] + dt * dl;
    y[SV_H] = x[SV_H] + dt * dh;
    y[SV_N] = x[SV_N] + dt * dn;
    y[SV_X] = x[SV_X] + dt * dx;
}

// Axon part: y[Va, ha, xa].
__device__ __forceinline__ void cell_step_axon(const CellParams& p, const float* __restrict__ x, float dt,
                                               float* __restrict__ y) {
    const float vs = x[SV_VS], va = x[SV_VA];

    // Axon: Na (instantaneous m^3, h), K (x^4), leak, coupling to the soma.
    const float ma = boltz(va, -30.0f, 5.5f);
    const float inaa = p.gNaA * ma * ma * ma * x[SV_HA] * (va - p.eNa);
    const float xa2 = x[SV_XA] * x[SV_XA];
    const float ika = p.gKA * xa2 * xa2 * (va - p.eK);
    const float ila = p.gLa * (va - p.eL);
    const float ias = p.gInt / p.p2 * (va - vs);
    const float dva = -(ika + ila + inaa + ias);

    const float tauha = 1.5f * expf(-(va + 40.0f) / 33.0f);
    const float dha = (boltz(va, -60.0f, -5.8f) - x[SV_HA]) / tauha;
    const float axa = 0.13f * ratio_expm1(-(va + 25.0f), 10.0f);
    const float bxa = 1.69f * expf(-0.0125f * (va + 35.0f));
    const float dxa = axa - (axa + bxa) * x[SV_XA];

    y[SV_VA] = va + dt * dva;
    y[SV_HA] = x[SV_HA] + dt * dha;
    y[SV_XA] = x[SV_XA] + dt * dxa;
}

// Next state of one cell. x: previous state, igap: gap current leaving the
// dendrite, iapp: evoked input into the dendrite, dt in ms.
__device__ __forceinline__ void cell_step(const CellParams& p, const float* __restrict__ x,
                                          float igap, float iapp, float dt,
                                          float* __restrict__ y) {
    cell_step_dendrite(p, x, igap, iapp, dt, y);
    cell_step_soma(p, x, dt, y);
    cell_step_axon(p, x, dt, y);
}

}  // namespace infoli
