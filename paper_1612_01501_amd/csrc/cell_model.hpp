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

// Floating-point contraction inside the compartment functions is limited
// to single expressions (the pragma below), so a cell's arithmetic is the
// same in every kernel that inlines it; the Euler updates are explicit
// fused multiply-adds.
//
// Arithmetic. Every exponential has an argument affine in one voltage,
// written (v - v0) * a: it is evaluated as 2^((v - v0) * a log2 e) on the
// transcendental unit (v_exp_f32, 1 ulp) with log2 e folded into the
// constant at compile time; the subtraction first keeps the argument's
// rounding relative to its own size. Divisions by a variable are a
// reciprocal (v_rcp_f32, 1 ulp) and a multiply, by a constant a multiply by
// its rounded reciprocal. Each result lies within a few ulp of the
// correctly rounded one.
constexpr double kLog2e = 1.4426950408889634074;

// a log2(e), rounded once to fp32 (folded where a is a constant)
__device__ __forceinline__ constexpr float l2(double a) { return float(a * kLog2e); }

__device__ __forceinline__ float ex2(float t) { return __builtin_amdgcn_exp2f(t); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// exp((v - v0) * a), c = l2(a)
__device__ __forceinline__ float exp_aff(float v, float v0, float c) { return ex2((v - v0) * c); }

// Steady-state curve 1/(1 + exp(-(v - vh)/k)); c = l2(-1/k), k < 0 for
// inactivation.
__device__ __forceinline__ float boltz(float v, float vh, float c) {
    return rcp(1.0f + exp_aff(v, vh, c));
}

// x / (exp(x/s) - 1) = s g(u), u = x/s, g(u) = u / (e^u - 1), continuous at
// u = 0 where g = 1. For |u| < 1/2, g is its Bernoulli series
// 1 - u/2 + u^2/12 - u^4/720 + u^6/30240 - u^8/1209600 (the next term is
// below 1e-10 there), which avoids the cancellation in e^u - 1; else the
// quotient itself.
__device__ __forceinline__ float ratio_expm1(float x, float s) {
    const float u = x * (1.0f / s);
    const float u2 = u * u;
    float q = fmaf(u2, -1.0f / 1209600.0f, 1.0f / 30240.0f);
    q = fmaf(u2, q, -1.0f / 720.0f);
    q = fmaf(u2, q, 1.0f / 12.0f);
    const float series = fmaf(u2, q, fmaf(u, -0.5f, 1.0f));
    const float direct = u * rcp(ex2(u * float(kLog2e)) - 1.0f);
    return s * (fabsf(u) < 0.5f ? series : direct);
}

// The update is Jacobi (every derivative from the previous-step state), so
// each compartment's next state is a function of x alone; the three parts
// below write disjoint entries of y and together are cell_step.

// Dendrite part: y[Vd, Ca, r, s, q]. igap: gap current leaving the dendrite,
// iapp: evoked input into the dendrite, dt in ms.
__device__ __forceinline__ void cell_step_dendrite(const CellParams& p, const float* __restrict__ x,
                                                   float igap, float iapp, float dt, float* __restrict__ y) {
#pragma clang fp contract(on)
    const float vd = x[SV_VD], vs = x[SV_VS];

    // Dendrite: high-threshold Ca (r^2), Ca-activated K (s), h current (q),
    // leak, coupling to the soma, gap junctions and the evoked input.
    // (each current's conductance factor times its driving force, the net
    // current accumulated with fused multiply-adds)
    const float icah = p.gCaH * x[SV_R] * x[SV_R] * (vd - p.eCa);
    float dvd = iapp - igap - icah;
    dvd = fmaf(-(p.gInt * rcp(1.0f - p.p1)), vd - vs, dvd);       // to the soma
    dvd = fmaf(-(p.gKCa * x[SV_S]), vd - p.eK, dvd);                // Ca-activated K
    dvd = fmaf(-(p.gH * x[SV_Q]), vd - p.eH, dvd);                  // h current
    dvd = fmaf(-p.gLd, vd - p.eL, dvd);                             // leak

    const float dca = fmaf(-3.0f, icah, -0.075f * x[SV_CA]);

    const float ar = 1.7f * boltz(vd, 5.0f, l2(-1.0 / 13.9));
    const float br = 0.02f * ratio_expm1(vd + 8.5f, 5.0f);
    const float dr = (ar - (ar + br) * x[SV_R]) * 0.2f;                  // tau_r = 5 ms

    const float as = fminf(0.00002f * x[SV_CA], 0.01f);
    const float ds = as - (as + 0.015f) * x[SV_S];

    const float qinf = boltz(vd, -80.0f, l2(1.0 / 4.0));
    // 1/tau_q = exp(-0.086 vd - 14.6) + exp(0.070 vd - 1.87)
    const float rq = exp_aff(vd, float(-14.6 / 0.086), l2(-0.086)) + exp_aff(vd, float(1.87 / 0.070), l2(0.070));
    const float dq = (qinf - x[SV_Q]) * rq;

    // C_m = 1 uF/cm^2: dV/dt equals the net inward current density.
    y[SV_VD] = fmaf(dt, dvd, vd);
    y[SV_CA] = fmaf(dt, dca, x[SV_CA]);
    y[SV_R] = fmaf(dt, dr, x[SV_R]);
    y[SV_S] = fmaf(dt, ds, x[SV_S]);
    y[SV_Q] = fmaf(dt, dq, x[SV_Q]);
}

// Soma part: y[Vs, k, l, h, n, x].
__device__ __forceinline__ void cell_step_soma(const CellParams& p, const float* __restrict__ x, float dt,
                                               float* __restrict__ y) {
#pragma clang fp contract(on)
    const float vd = x[SV_VD], vs = x[SV_VS], va = x[SV_VA];

    // Soma: low-threshold Ca (k^3 l), Na (instantaneous m^3, h), delayed
    // rectifier K (n^4), K (x^4), leak, coupling to dendrite and axon.
    const float kk = x[SV_K];
    const float ms = boltz(vs, -30.0f, l2(-1.0 / 5.5));
    const float n2 = x[SV_N] * x[SV_N];
    const float x2 = x[SV_X] * x[SV_X];
    float dvs = -(p.gCaL * kk * kk * kk * x[SV_L]) * (vs - p.eCa);   // low-threshold Ca
    dvs = fmaf(-(p.gNaS * ms * ms * ms * x[SV_H]), vs - p.eNa, dvs);  // Na
    dvs = fmaf(-(p.gKdrS * n2 * n2 + p.gKS * x2 * x2), vs - p.eK, dvs); // delayed rectifier K, K
    dvs = fmaf(-p.gLs, vs - p.eL, dvs);                                // leak
    dvs = fmaf(-(p.gInt * rcp(p.p1)), vs - vd, dvs);                   // to the dendrite
    dvs = fmaf(-(p.gInt * rcp(1.0f - p.p2)), vs - va, dvs);            // to the axon

    const float dk = boltz(vs, -61.0f, l2(-1.0 / 4.2)) - kk;              // tau_k = 1 ms
    // tau_l = 20 e1 / (1 + e2) + 35, e1 = exp((vs + 160)/30), e2 = exp((vs + 84)/7.3):
    // 1/tau_l = (1 + e2) / (20 e1 + 35 (1 + e2))
    const float e1 = exp_aff(vs, -160.0f, l2(1.0 / 30.0));
    const float e2p1 = 1.0f + exp_aff(vs, -84.0f, l2(1.0 / 7.3));
    const float dl = (boltz(vs, -85.5f, l2(1.0 / 8.5)) - x[SV_L]) * e2p1 * rcp(fmaf(20.0f, e1, 35.0f * e2p1));
    // tau_h = 3 exp(-(vs + 40)/33): 1/tau_h = exp((vs + 40)/33) / 3
    const float dh = (boltz(vs, -70.0f, l2(1.0 / 5.8)) - x[SV_H]) * (exp_aff(vs, -40.0f, l2(1.0 / 33.0)) * (1.0f / 3.0f));
    const float taun = fmaf(47.0f, exp_aff(vs, -50.0f, l2(1.0 / 900.0)), 5.0f);
    const float dn = (boltz(vs, -3.0f, l2(-1.0 / 10.0)) - x[SV_N]) * rcp(taun);
    const float axs = 0.13f * ratio_expm1(-(vs + 25.0f), 10.0f);
    const float bxs = 1.69f * exp_aff(vs, -35.0f, l2(-0.0125));
    const float dx = axs - (axs + bxs) * x[SV_X];

    y[SV_VS] = fmaf(dt, dvs, vs);
    y[SV_K] = fmaf(dt, dk, kk);
    y[SV_L] = fmaf(dt, dl, x[SV_L]);
    y[SV_H] = fmaf(dt, dh, x[SV_H]);
    y[SV_N] = fmaf(dt, dn, x[SV_N]);
    y[SV_X] = fmaf(dt, dx, x[SV_X]);
}

// Axon part: y[Va, ha, xa].
__device__ __forceinline__ void cell_step_axon(const CellParams& p, const float* __restrict__ x, float dt,
                                               float* __restrict__ y) {
#pragma clang fp contract(on)
    const float vs = x[SV_VS], va = x[SV_VA];

    // Axon: Na (instantaneous m^3, h), K (x^4), leak, coupling to the soma.
    const float ma = boltz(va, -30.0f, l2(-1.0 / 5.5));
    const float xa2 = x[SV_XA] * x[SV_XA];
    float dva = -(p.gKA * xa2 * xa2) * (va - p.eK);                    // K
    dva = fmaf(-p.gLa, va - p.eL, dva);                                // leak
    dva = fmaf(-(p.gNaA * ma * ma * ma * x[SV_HA]), va - p.eNa, dva);  // Na
    dva = fmaf(-(p.gInt * rcp(p.p2)), va - vs, dva);                   // to the soma

    // tau_ha = 1.5 exp(-(va + 40)/33): 1/tau_ha = exp((va + 40)/33) / 1.5
    const float dha = (boltz(va, -60.0f, l2(1.0 / 5.8)) - x[SV_HA]) * (exp_aff(va, -40.0f, l2(1.0 / 33.0)) * (1.0f / 1.5f));
    const float axa = 0.13f * ratio_expm1(-(va + 25.0f), 10.0f);
    const float bxa = 1.69f * exp_aff(va, -35.0f, l2(-0.0125));
    const float dxa = axa - (axa + bxa) * x[SV_XA];

    y[SV_VA] = fmaf(dt, dva, va);
    y[SV_HA] = fmaf(dt, dha, x[SV_HA]);
    y[SV_XA] = fmaf(dt, dxa, x[SV_XA]);
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
