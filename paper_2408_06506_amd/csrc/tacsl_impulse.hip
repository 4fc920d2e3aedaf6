// Batched implicit soft-contact impulse (Section III-A, "Constraint
// Solution"), one contact per element, over every contact of every
// environment at once.
//
// The contact force is the Kelvin-Voigt law max(-kappa eps - c eps_dot, 0)
// imposed at the end of the step (implicit spring); with the semi-implicit
// Euler update and lambda = m * (change of eps_dot), the impulse has the
// closed form of the paper's contact-impulse equation:
//   alpha  = dt (dt kappa + c)
//   lambda = max(0, (-dt kappa eps - alpha eps_dot) / (1 + alpha / m))
//   dv     = lambda / m.
// The work is a pure stream (16 bytes read, 8 written per contact), so the
// kernel is written for HBM: 16-byte loads of four contacts per lane,
// non-temporal loads and stores, one grid step per lane (a wider grid keeps
// more bytes in flight than a chip-sized grid-stride loop: 6.1 vs 5.8 TB/s on
// a 33.5 M-contact stream), and one atomic per wavefront for the rare invalid
// contact.
#include <cstdint>
#include <cmath>

#include <hip/hip_runtime.h>

#include "tacsl.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef int32_t v4i __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
constexpr int kMaxGrid = 1 << 20;  // one grid step per lane up to 2^28 lanes; the loop covers the rest

struct Contact {
  float lambda, dv;
  bool bad;
};

__device__ __forceinline__ Contact impulse(float eps, float eps_dot, float inv_mass, float kappa, float c, float dt) {
  const float alpha = dt * fmaf(dt, kappa, c);
  const float num = -(dt * kappa) * eps - alpha * eps_dot;
  const float den = fmaf(alpha, inv_mass, 1.0f);
  const float l = num / den;
  Contact r;
  // invalid: non-finite input or result, or a non-positive denominator (negative 1/m)
  r.bad = !(den > 0.0f && den < INFINITY && fabsf(l) < INFINITY);
  r.lambda = (!r.bad && l > 0.0f) ? l : 0.0f;
  r.dv = r.bad ? 0.0f : r.lambda * inv_mass;  // 0 * inf would be NaN
  return r;
}

__device__ __forceinline__ float2 env_constants(const float2* __restrict__ kc, const int32_t* __restrict__ env,
                                                int64_t k, int32_t n_env, bool& bad) {
  if (!env) return kc[0];
  const int32_t e = __builtin_nontemporal_load(env + k);
  if (e < 0 || e >= n_env) {
    bad = true;
    return make_float2(0.0f, 0.0f);
  }
  return kc[e];
}

__device__ __forceinline__ void flag_wave(bool bad, uint32_t* status) {
  const uint64_t m = __ballot(bad);
  if (m && status && (threadIdx.x & 63u) == (uint32_t)(__ffsll((unsigned long long)m) - 1))
    atomicOr(status, (uint32_t)TACSL_DEV_BAD_CONTACT);
}

// Four contacts per lane with 16-byte accesses; every pointer 16-byte aligned.
__global__ __launch_bounds__(kBlock) void k_contact_impulse_x4(
    const v4f* __restrict__ eps, const v4f* __restrict__ eps_dot, const v4f* __restrict__ inv_mass,
    const v4i* __restrict__ env, const float2* __restrict__ kc, int32_t n_env, float dt,
    v4f* __restrict__ lambda, v4f* __restrict__ dv, uint32_t* status, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n4; q += stride) {
    const v4f e = __builtin_nontemporal_load(eps + q);
    const v4f ed = __builtin_nontemporal_load(eps_dot + q);
    const v4f im = __builtin_nontemporal_load(inv_mass + q);
    float2 p[4];
    bool bad = false;
    if (env) {
      const v4i ev = __builtin_nontemporal_load(env + q);
      const int32_t ei[4] = {ev.x, ev.y, ev.z, ev.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool in = ei[j] >= 0 && ei[j] < n_env;
        bad |= !in;
        const float2 v = kc[in ? ei[j] : 0];
        p[j] = in ? v : make_float2(NAN, NAN);  // NaN constants mark the contact invalid below
      }
    } else {
      p[0] = p[1] = p[2] = p[3] = kc[0];
    }
    const Contact c0 = impulse(e.x, ed.x, im.x, p[0].x, p[0].y, dt);
    const Contact c1 = impulse(e.y, ed.y, im.y, p[1].x, p[1].y, dt);
    const Contact c2 = impulse(e.z, ed.z, im.z, p[2].x, p[2].y, dt);
    const Contact c3 = impulse(e.w, ed.w, im.w, p[3].x, p[3].y, dt);
    bad |= c0.bad | c1.bad | c2.bad | c3.bad;
    __builtin_nontemporal_store(v4f{c0.lambda, c1.lambda, c2.lambda, c3.lambda}, lambda + q);
    if (dv) __builtin_nontemporal_store(v4f{c0.dv, c1.dv, c2.dv, c3.dv}, dv + q);
    flag_wave(bad, status);
  }
}

// One contact per lane: the tail of the x4 kernel, or any alignment.
__global__ __launch_bounds__(kBlock) void k_contact_impulse_x1(
    const float* __restrict__ eps, const float* __restrict__ eps_dot, const float* __restrict__ inv_mass,
    const int32_t* __restrict__ env, const float2* __restrict__ kc, int32_t n_env, float dt,
    float* __restrict__ lambda, float* __restrict__ dv, uint32_t* status, int64_t k0, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = k0 + (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) {
    bool bad = false;
    const float2 p = env_constants(kc, env, k, n_env, bad);
    const Contact c = bad ? Contact{0.0f, 0.0f, true}
                          : impulse(__builtin_nontemporal_load(eps + k), __builtin_nontemporal_load(eps_dot + k),
                                    __builtin_nontemporal_load(inv_mass + k), p.x, p.y, dt);
    __builtin_nontemporal_store(c.lambda, lambda + k);
    if (dv) __builtin_nontemporal_store(c.dv, dv + k);
    flag_wave(c.bad, status);
  }
}

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

inline int grid_for(int64_t work) {
  const int64_t g = (work + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > kMaxGrid ? kMaxGrid : g));
}

}  // namespace

extern "C" int tacsl_contact_impulse(int64_t n, const float* eps, const float* eps_dot, const float* inv_mass,
                                     const int32_t* env, int32_t n_env, const float* kc, float dt, float* lambda,
                                     float* dv, uint32_t* status, hipStream_t stream) {
  if (n < 0 || n_env < 1) return TACSL_ERR_SHAPE;
  if (!(dt > 0.0f) || !std::isfinite(dt)) return TACSL_ERR_RANGE;
  if (n == 0) return TACSL_OK;
  if (!eps || !eps_dot || !inv_mass || !kc || !lambda) return TACSL_ERR_NULL_ARG;
  if (((uintptr_t)kc & 7u) != 0) return TACSL_ERR_RANGE;
  const float2* kc2 = reinterpret_cast<const float2*>(kc);
  const bool vec = aligned16(eps) && aligned16(eps_dot) && aligned16(inv_mass) && aligned16(lambda) &&
                   (!env || aligned16(env)) && (!dv || aligned16(dv));
  int64_t done = 0;
  if (vec && n >= 4) {
    const int64_t n4 = n / 4;
    hipLaunchKernelGGL(k_contact_impulse_x4, dim3(grid_for(n4)), dim3(kBlock), 0, stream,
                       reinterpret_cast<const v4f*>(eps), reinterpret_cast<const v4f*>(eps_dot),
                       reinterpret_cast<const v4f*>(inv_mass), reinterpret_cast<const v4i*>(env), kc2, n_env, dt,
                       reinterpret_cast<v4f*>(lambda), reinterpret_cast<v4f*>(dv), status, n4);
    if (hipGetLastError() != hipSuccess) return TACSL_ERR_HIP;
    done = n4 * 4;
  }
  if (done < n) {
    hipLaunchKernelGGL(k_contact_impulse_x1, dim3(grid_for(n - done)), dim3(kBlock), 0, stream, eps, eps_dot,
                       inv_mass, env, kc2, n_env, dt, lambda, dv, status, done, n);
    if (hipGetLastError() != hipSuccess) return TACSL_ERR_HIP;
  }
  return TACSL_OK;
}
