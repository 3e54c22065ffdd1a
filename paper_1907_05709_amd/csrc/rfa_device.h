// rfa_device.h -- device-side definitions shared by the stepper kernels.
//
// The state is the excess temperature theta = T - 37 degC held as an
// unevaluated float-float pair (hi, lo): plain FP32 cannot keep the explicit
// update's rounding below 1e-4 K at the 700-1500 degC needle-axis
// temperatures of Gaussian line sources of tens of watts, while the pair
// carries ~48 bits.  Coefficient tables are float-float as well (their
// FP32 rounding is coherent over a whole region and would bias the result
// by ~1 ulp of the peak temperature).  The source increment is FP32.
//
// Voxel update (Eq. (CUDAbioheat3d) with per-class conductivity in flux form,
// Alg. 1 for held voxels), in excess temperature:
//   theta' = theta + sum_axes [C(l,l-)(theta- - theta) + C(l,l+)(theta+ - theta)]
//                  - B_l f_p g_p theta + Qs_l + s_p
// with C(a,b) = dt K_face(a,b) / (rho_a c_a d^2), K_face the harmonic mean,
// B_l = dt h_l / (rho_l c_l), Qs_l = dt (Q_l + h_l (T_a - 37)) / (rho_l c_l),
// s_p = dt q_p / (rho c) the RF increment, f_p the optional perfusion
// multiplier and g_p = exp(-Omega_p) the surviving cell fraction when the
// perfusion is damage-coupled (Linte's tissue-state factor, Eq.
// (2675-eq1_Linte) with Omega = ln(c(0)/c(t)) of Eq. (eq-tissState); Omega
// at the start of the step), else 1.  Damage (Eq. (eq-tissState), T in Kelvin, left point):
//   Omega' = min(Omega + dt k_a exp(min(c theta / (T_aK + theta), 80)), cap)
// with T_aK = 310.15 K, k_a = A exp(-Ea / (R T_aK)), c = Ea / (R T_aK).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rfa {

// Internal label byte: class index in bits 3-6, flags in bits 0, 1, 2 and 7.
// With the class stored times 8, lab & kClassMask is the byte offset of the
// class's float2 entry in a row of a coefficient table.
constexpr unsigned kClassShift = 3;
constexpr unsigned kClassMask = 0x78u;  // class << kClassShift
constexpr unsigned kTissue = 0x01u;     // class accumulates damage
constexpr unsigned kHeld = 0x02u;       // fixed class or outermost layer
constexpr unsigned kSource = 0x04u;     // RF increment s != 0 (s is read only there)
constexpr unsigned kLatch = 0x80u;      // t_death reached (sticky)
constexpr int kMaxClasses = 16;

__host__ __device__ constexpr unsigned class_of(unsigned lab) {
  return (lab & kClassMask) >> kClassShift;
}

// Per-dt coefficient tables, staged into LDS by every work-group.
struct Tables {
  float2 cf[3][kMaxClasses * kMaxClasses];  // [axis][a*16+b] = C(a,b) hi/lo
  float4 cls[kMaxClasses];                  // {B hi, B lo, Qs, rho c V}
};

// Damage / latch constants of one dt.
struct StepConst {
  float dtka;    // dt * k_a
  float c2;      // c * log2(e)
  float tak;     // T_aK = 310.15
  float clamp2;  // 80 * log2(e)
  float cap;     // Omega cap
  float thr;     // t_death - 37
  float decay2;  // log2(e) with damage-coupled perfusion, else 0
};

// Per-thread diagnostic partials of one step.
struct Partial {
  float perf;     // sum rho c V * (B f theta)       -> J removed by perfusion
  float bnd;      // sum rho c V * conduction term   -> J received from held voxels
  unsigned mono;  // free voxels that cooled by more than kCoolRel |theta| + kCoolAbs
};

// The cooling-voxel count takes a free voxel as cooling when its increment
// is below -(kCoolRel |theta| + kCoolAbs).  The increment's FP32 rounding
// error is about 10 eps (sum_faces C |d| +
// |B f theta| + |Qs + s|) (six chained face terms, the float-float
// differences, the sink, the final sums); where the increment is near zero
// (conduction, perfusion and source in balance, near the steady state)
// those magnitudes are at most about 2 |theta| below the step bound, so a
// smaller fall has an undetermined sign.  kCoolRel = 64 eps leaves a margin
// of three.  In the far field the temperature excess decays into FP32's
// subnormal range, where the spacing is absolute (1.4e-45) and the relative
// bound fails; falls below kCoolAbs = 1e-30 K are not counted either.
constexpr float kCoolRel = 64.0f / 16777216.0f;  // 2^-18
constexpr float kCoolAbs = 1e-30f;                // K

// Float-float difference theta_nb - theta, rounded once.
__device__ __forceinline__ float ff_diff(float hn, float ln, float hi, float lo) {
  return (hn - hi) + (ln - lo);
}

// One voxel of one step.  No output of a held voxel depends on its
// neighbours' values, which may be arbitrary (even NaN: the tiled kernels
// leave halo cells outside the grid unwritten), so those values only ever
// reach results through selects on the held flag.
// cf points at the LDS copy of Tables::cf (3 x 256 float2), cls at Tables::cls.
//
// The damage update has two forms with the same bits: branch-free (the
// default, one basic block per plane, fewer live registers in the kernels
// with one or two voxels per lane) and a select that lets the compiler
// branch around the transcendentals off tissue (kSelectDamage, fewer live
// registers where each lane carries four voxels).
//
// field: pf comes from a perfusion field (kernels with a field; a constant
// after inlining).  Only those kernels apply the damage coupling: the host
// gives every damage-coupled grid a field (all ones if none was set).  With
// the coupling off (K.decay2 = 0) the factor is exp2(-0) = 1 and pf * 1 = pf
// exactly, for every finite om >= 0 (callers pass a finite damage integral,
// also into scratch recomputations).
template <bool kSelectDamage = false>
__device__ __forceinline__ void voxel_step(
    float hi, float lo, unsigned lab,
    float hxm, float lxm, unsigned bxm, float hxp, float lxp, unsigned bxp,
    float hym, float lym, unsigned bym, float hyp, float lyp, unsigned byp,
    float hzm, float lzm, unsigned bzm, float hzp, float lzp, unsigned bzp,
    float s, float pf, float& om, const float2* __restrict__ cf,
    const float4* __restrict__ cls, const StepConst& K,
    float& nh, float& nl, unsigned& nlab, Partial& acc, bool field = false) {
  if (field) pf *= __builtin_amdgcn_exp2f(-om * K.decay2);
  // C(l, l_nb) addressed in bytes: row of the own class (16 entries of 8
  // bytes), entry of the neighbour's class (its masked label byte)
  const unsigned row = (lab & kClassMask) << 4;
  auto entry = [&](int axis, unsigned nb) {
    const char* t = reinterpret_cast<const char*>(cf + axis * kMaxClasses * kMaxClasses);
    return *reinterpret_cast<const float2*>(t + (row | (nb & kClassMask)));
  };
  const float2 kxm = entry(0, bxm), kxp = entry(0, bxp);
  const float2 kym = entry(1, bym), kyp = entry(1, byp);
  const float2 kzm = entry(2, bzm), kzp = entry(2, bzp);
  const float dxm = ff_diff(hxm, lxm, hi, lo), dxp = ff_diff(hxp, lxp, hi, lo);
  const float dym = ff_diff(hym, lym, hi, lo), dyp = ff_diff(hyp, lyp, hi, lo);
  const float dzm = ff_diff(hzm, lzm, hi, lo), dzp = ff_diff(hzp, lzp, hi, lo);
  // Six face terms C(l, l_nb) d_nb, one fused chain per part of the
  // float-float coefficient (the lo chain carries the coefficients'
  // rounding, which is the same over a whole region).
  float ch = kxm.x * dxm, cl = kxm.y * dxm;
  ch = __builtin_fmaf(kxp.x, dxp, ch);
  cl = __builtin_fmaf(kxp.y, dxp, cl);
  ch = __builtin_fmaf(kym.x, dym, ch);
  cl = __builtin_fmaf(kym.y, dym, cl);
  ch = __builtin_fmaf(kyp.x, dyp, ch);
  cl = __builtin_fmaf(kyp.y, dyp, cl);
  ch = __builtin_fmaf(kzm.x, dzm, ch);
  cl = __builtin_fmaf(kzm.y, dzm, cl);
  ch = __builtin_fmaf(kzp.x, dzp, ch);
  cl = __builtin_fmaf(kzp.y, dzp, cl);
  const float cond = ch + cl;
  const float4 c = cls[class_of(lab)];
  const float bh = c.x * pf, bl = c.y * pf;
  const float perf = __builtin_fmaf(bh, hi, __builtin_fmaf(bl, hi, bh * lo));
  const float inc = (cond - perf) + (c.z + s);
  // float-float accumulation: (hi, lo) + inc, renormalised
  const float t = lo + inc;
  const float s1 = hi + t;
  const float v = s1 - hi;
  const float e = (hi - (s1 - v)) + (t - v);
  const float h2 = s1 + e;
  const float l2 = e - (h2 - s1);
  const bool held = (lab & kHeld) != 0u;
  nh = held ? hi : h2;
  nl = held ? lo : l2;
  // Arrhenius increment evaluated at the step's input temperature.
  float x = K.c2 * hi * __builtin_amdgcn_rcpf(K.tak + hi);
  x = fminf(x, K.clamp2);
  const float rate = K.dtka * __builtin_amdgcn_exp2f(x);
  const bool tissue = (lab & kTissue) != 0u;
  if constexpr (kSelectDamage) {
    om = tissue ? fminf(om + rate, K.cap) : om;
  } else {
    // off tissue: om + rate * 0 = om and fminf(om, inf) = om (om >= +0)
    om = fminf(__builtin_fmaf(rate, tissue ? 1.0f : 0.0f, om),
               tissue ? K.cap : __builtin_huge_valf());
  }
  const bool reached = (nh > K.thr) | ((nh == K.thr) & (nl >= 0.0f));
  nlab = (tissue && reached) ? (lab | kLatch) : lab;
  acc.mono += (!held && inc < -__builtin_fmaf(kCoolRel, fabsf(hi), kCoolAbs)) ? 1u : 0u;
  acc.perf = held ? acc.perf : __builtin_fmaf(c.w, perf, acc.perf);
  acc.bnd = held ? acc.bnd : __builtin_fmaf(c.w, cond, acc.bnd);
}

// Wave sums through DPP lane moves instead of LDS permutes: lanes ^ 1 and
// ^ 2 within quads, the half-row and row mirrors (every lane then holds its
// 16-lane row's sum), then the GFX9 row broadcasts (lane 15 of rows 0 and
// 2 added to rows 1 and 3, lane 31 to rows 2 and 3), which leave the total
// in lane 63; it is read back to every lane.  Six dependent VALU steps
// instead of six LDS round trips, in a fixed order.  Rows a move does not
// write receive 0 (the old operand).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kCtrl, kRowMask, 0xF, false);
}

template <typename T, typename Add>
__device__ __forceinline__ T wave_sum_dpp(T v, Add add) {
  auto bits = [](T x) { return __builtin_bit_cast(int, x); };
  auto val = [](int x) { return __builtin_bit_cast(T, x); };
  v = add(v, val(dpp_move<0xB1, 0xF>(bits(v))));   // quad_perm [1,0,3,2]
  v = add(v, val(dpp_move<0x4E, 0xF>(bits(v))));   // quad_perm [2,3,0,1]
  v = add(v, val(dpp_move<0x141, 0xF>(bits(v))));  // row_half_mirror
  v = add(v, val(dpp_move<0x140, 0xF>(bits(v))));  // row_mirror
  v = add(v, val(dpp_move<0x142, 0xA>(bits(v))));  // row_bcast:15 into rows 1, 3
  v = add(v, val(dpp_move<0x143, 0xC>(bits(v))));  // row_bcast:31 into rows 2, 3
  return val(__builtin_amdgcn_readlane(bits(v), 63));
}

__device__ __forceinline__ float wave_sum(float v) {
  return wave_sum_dpp(v, [](float a, float b) { return a + b; });
}

__device__ __forceinline__ unsigned wave_sum_u(unsigned v) {
  return wave_sum_dpp(v, [](unsigned a, unsigned b) { return a + b; });
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace rfa
