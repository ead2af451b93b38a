// Step rules shared by the SVGD update and the ADVI step: SGD, AdaGrad,
// AdaDelta and Adam (section 2.2 lists the four; the rules follow Duchi et al.
// 2011, Zeiler 2012 and Kingma & Ba 2014).  Each applies to one coordinate of
// an ascent direction with its own per-coordinate FP32 state.
#pragma once

#include <cmath>

#include "vip.h"

struct OptArgs {
  int kind = VIP_OPT_SGD;
  float *s1 = nullptr, *s2 = nullptr;
  float b1 = 0.f, b2 = 0.f, delta = 0.f;
  float c1 = 1.f, c2 = 1.f;   // Adam bias corrections 1 / (1 - b1^t), 1 / (1 - b2^t)
};
// The state of one coordinate in registers, so that a kernel can issue the
// loads of several coordinates before their arithmetic.
struct OptState {
  float a = 0.f, b = 0.f;
};
__device__ __forceinline__ OptState opt_load(const OptArgs &o, long long e) {
  OptState st;
  if (o.kind != VIP_OPT_SGD) st.a = o.s1[e];
  if (o.kind == VIP_OPT_ADADELTA || o.kind == VIP_OPT_ADAM) st.b = o.s2[e];
  return st;
}
__device__ __forceinline__ void opt_store(const OptArgs &o, long long e, const OptState &st) {
  if (o.kind != VIP_OPT_SGD) o.s1[e] = st.a;
  if (o.kind == VIP_OPT_ADADELTA || o.kind == VIP_OPT_ADAM) o.s2[e] = st.b;
}
// Increment for direction p; updates the state in place.
__device__ __forceinline__ float opt_apply(const OptArgs &o, OptState &st, float p, float eps) {
  switch (o.kind) {
    case VIP_OPT_ADAGRAD: {
      st.a = st.a + p * p;
      return eps * p / (sqrtf(st.a) + o.delta);
    }
    case VIP_OPT_ADADELTA: {
      const float Eg = o.b1 * st.a + (1.0f - o.b1) * p * p;
      const float Ed = st.b;
      const float u = sqrtf(Ed + o.delta) / sqrtf(Eg + o.delta) * p;
      st.a = Eg;
      st.b = o.b1 * Ed + (1.0f - o.b1) * u * u;
      return eps * u;
    }
    case VIP_OPT_ADAM: {
      const float mo = o.b1 * st.a + (1.0f - o.b1) * p;
      const float ve = o.b2 * st.b + (1.0f - o.b2) * p * p;
      st.a = mo;
      st.b = ve;
      return eps * (mo * o.c1) / (sqrtf(ve * o.c2) + o.delta);
    }
    default: return eps * p;
  }
}
__device__ __forceinline__ float opt_step(const OptArgs &o, long long e, float p, float eps) {
  OptState st = opt_load(o, e);
  const float inc = opt_apply(o, st, p, eps);
  opt_store(o, e, st);
  return inc;
}

// Checks a caller's step rule and converts it; NULL means plain SGD.
static inline vip_status make_opt_args(const vip_optimizer *opt, OptArgs *oa) {
  *oa = OptArgs{};
  if (!opt) return VIP_OK;
  if (opt->kind < VIP_OPT_SGD || opt->kind > VIP_OPT_ADAM) return VIP_E_ARG;
  const bool two = opt->kind == VIP_OPT_ADADELTA || opt->kind == VIP_OPT_ADAM;
  if (opt->kind != VIP_OPT_SGD && (!opt->s1 || (two && !opt->s2))) return VIP_E_ARG;
  if (opt->kind == VIP_OPT_ADAM && opt->t < 1) return VIP_E_ARG;
  if (!(opt->delta >= 0.0) || !(opt->beta1 >= 0.0 && opt->beta1 < 1.0) ||
      !(opt->beta2 >= 0.0 && opt->beta2 < 1.0))
    return VIP_E_ARG;
  oa->kind = opt->kind;
  oa->s1 = opt->s1;
  oa->s2 = opt->s2;
  oa->b1 = float(opt->beta1);
  oa->b2 = float(opt->beta2);
  oa->delta = float(opt->delta);
  if (opt->kind == VIP_OPT_ADAM) {
    oa->c1 = float(1.0 / (1.0 - std::pow(opt->beta1, double(opt->t))));
    oa->c2 = float(1.0 / (1.0 - std::pow(opt->beta2, double(opt->t))));
  }
  return VIP_OK;
}
