// Device-side building blocks of one MPPI iteration (gfx950).
//
// Noise: Philox4x64-10 (Salmon et al., SC'11) keyed by (seed, 0) with
// counter (k, t, instance, tick); each 64-bit word yields one uniform from
// its top 23 bits, Box-Muller (1958) turns two uniforms into two normals.
// Dynamics: collective thrust + body rates, attitude held over the step for
// the acceleration, exact exponential map for the attitude (Section IV-A uses
// a standard quadrotor model; the input form is this library's reading).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "solve_desc.hpp"
#include "weights.hpp"

namespace mppi {

// ---------------------------------------------------------------- Philox4x64-10
struct u64x4 { uint64_t x0, x1, x2, x3; };

__device__ __forceinline__ u64x4 philox4x64_10(u64x4 c, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c.x0), lo0 = M0 * c.x0;
    const uint64_t hi1 = __umul64hi(M1, c.x2), lo1 = M1 * c.x2;
    c = u64x4{hi1 ^ c.x1 ^ k0, lo1, hi0 ^ c.x3 ^ k1, lo0};
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// Top 23 bits -> (m + 1/2) 2^-23, exact in float32, strictly inside (0, 1).
__device__ __forceinline__ float uniform23(uint64_t w) {
  return ((float)(uint32_t)(w >> 41) + 0.5f) * 0x1.0p-23f;
}

// Four standard normals for (rollout k, step t) of a solve.
__device__ __forceinline__ void normals4(uint64_t seed, uint64_t inst, uint64_t tick, uint32_t k,
                                         uint32_t t, float n[4]) {
  const u64x4 w = philox4x64_10(u64x4{k, t, inst, tick}, seed, 0ull);
  const float u0 = uniform23(w.x0), u1 = uniform23(w.x1);
  const float u2 = uniform23(w.x2), u3 = uniform23(w.x3);
  const float r01 = sqrtf(-2.0f * logf(u0));
  const float r23 = sqrtf(-2.0f * logf(u2));
  float s, c;
  sincospif(2.0f * u1, &s, &c);
  n[0] = r01 * c;
  n[1] = r01 * s;
  sincospif(2.0f * u3, &s, &c);
  n[2] = r23 * c;
  n[3] = r23 * s;
}

// u = clip(U_nom[t] + L n, lo, hi) with L lower triangular (row-major 4x4).
__device__ __forceinline__ void sample_control(const SolveDesc& d, uint32_t k, uint32_t t,
                                               uint64_t tick, float u[4]) {
  float n[4];
  normals4(d.seed, d.instance_id, tick, k, t, n);
  const int ti = t < (uint32_t)d.U_len ? (int)t : d.U_len - 1;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float e = 0.0f;
#pragma unroll
    for (int j = 0; j <= c; ++j) e = fmaf(d.L[c * 4 + j], n[j], e);
    const float nom = d.U_src ? (float)d.U_src[ti * 4 + c] : (float)d.hover[c];
    u[c] = fminf(fmaxf(nom + e, d.u_lo[c]), d.u_hi[c]);
  }
}

// ---------------------------------------------------------------- latent fold
// c_g = W1[:, 3:] z_g + b1 for gate g of solve d, in FP64 and rounded once:
// the decoder's first layer applied to the latent block of its input [p; z]
// (Section III-B), shared by all queries of a gate.  With an instance cache
// (object permanence, Section IV-B-3) an observed gate's fold is also stored
// there, and an unobserved gate's fold is taken from it.  One workgroup per
// gate (any size).
__device__ __forceinline__ void fold_gate(const SolveDesc& d, int g, const DeviceWeights& w) {
  if (g >= d.G || d.sdf_kind != 0) return;
  float* cache = d.cf_cache ? d.cf_cache + (size_t)g * d.H : nullptr;
  if ((d.fold_cached >> g) & 1u) {
    for (int m = threadIdx.x; m < d.H; m += blockDim.x) d.cfold[g * d.H + m] = cache[m];
    return;
  }
  const float* z = d.z + g * kLatent;
  for (int m = threadIdx.x; m < d.H; m += blockDim.x) {
    // (the transposed block: neighbouring threads read neighbouring words;
    // all 64 reads go out before the first product, one memory latency)
    double wv[kLatent];
#pragma unroll
    for (int j = 0; j < kLatent; ++j) wv[j] = w.w0lat[(size_t)j * d.H + m];
    double acc = w.b0[m];
#pragma unroll
    for (int j = 0; j < kLatent; ++j) acc = fma(wv[j], (double)z[j], acc);
    d.cfold[g * d.H + m] = (float)acc;
    if (cache) cache[m] = (float)acc;
  }
}

// ---------------------------------------------------------------- dynamics
// Rollout state in the local frame: dp is the position minus p0 + v0 t dt
// (deviation from the initial ballistic drift), dv = v - v0, q attitude.
struct RolloutState {
  float dp[3], dv[3], q[4];
};

// Attitude increment of one step from the body rate (u[1], u[2], u[3]):
// r = [cos(|w| dt/2), sin(|w| dt/2) w/|w|].  It depends on the input only,
// so a rollout loop may form it ahead of the state update.  Two parts: the
// Taylor series in (|w| dt/2)^2 for every lane (branch-free, truncation
// < 3e-13 below 1/4: no division, no range reduction), then sincos for the
// lanes at or above 1/4.
__device__ __forceinline__ float quad_rotation_series(const float u[4], float dt, float r[4]) {
  const float wx = u[1], wy = u[2], wz = u[3];
  const float nrm = sqrtf(wx * wx + wy * wy + wz * wz);
  const float half = 0.5f * nrm * dt;
  const float x2 = half * half;
  const float ch = fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, 1.0f / 40320.0f, -1.0f / 720.0f), 1.0f / 24.0f), -0.5f), 1.0f);
  const float so = 0.5f * dt *
      fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, 1.0f / 362880.0f, -1.0f / 5040.0f), 1.0f / 120.0f), -1.0f / 6.0f), 1.0f);
  r[0] = ch;
  r[1] = so * wx;
  r[2] = so * wy;
  r[3] = so * wz;
  return half;
}
__device__ __forceinline__ void quad_rotation_large(const float u[4], float half, float r[4]) {
  if (half >= 0.25f) {
    const float wx = u[1], wy = u[2], wz = u[3];
    const float nrm = sqrtf(wx * wx + wy * wy + wz * wz);
    float sh, ch;
    sincosf(half, &sh, &ch);
    const float so = sh / nrm;
    r[0] = ch;
    r[1] = so * wx;
    r[2] = so * wy;
    r[3] = so * wz;
  }
}
__device__ __forceinline__ void quad_rotation(const float u[4], float dt, float r[4]) {
  quad_rotation_large(u, quad_rotation_series(u, dt, r), r);
}

// One step of the state with collective thrust f_c = u0 and the attitude
// increment r of quad_rotation: position and velocity from the thrust along
// the body z axis and gravity, then q <- q (x) r.
__device__ __forceinline__ void quad_advance(RolloutState& s, float u0, const float r[4], float dt, float inv_m,
                                             float g) {
  const float w = s.q[0], x = s.q[1], y = s.q[2], z = s.q[3];
  // R(q) e3: body z axis in the world frame.
  const float bx = 2.0f * (x * z + w * y);
  const float by = 2.0f * (y * z - w * x);
  const float bz = 1.0f - 2.0f * (x * x + y * y);
  const float f = u0 * inv_m;
  const float a[3] = {f * bx, f * by, fmaf(f, bz, -g)};
  const float hdt2 = 0.5f * dt * dt;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s.dp[i] = fmaf(a[i], hdt2, fmaf(s.dv[i], dt, s.dp[i]));
    s.dv[i] = fmaf(a[i], dt, s.dv[i]);
  }
  const float rw = r[0], rx = r[1], ry = r[2], rz = r[3];
  s.q[0] = w * rw - x * rx - y * ry - z * rz;
  s.q[1] = w * rx + x * rw + y * rz - z * ry;
  s.q[2] = w * ry - x * rz + y * rw + z * rx;
  s.q[3] = w * rz + x * ry - y * rx + z * rw;
}

__device__ __forceinline__ void quad_step(RolloutState& s, const float u[4], float dt, float inv_m,
                                          float g) {
  float r[4];
  quad_rotation(u, dt, r);
  quad_advance(s, u[0], r, dt, inv_m, g);
}

// Rotor-thrust-rate input (Section IV-A): the four rotor thrusts and the
// body rate are state.  One step: thrusts integrate their rates and are
// clipped to [0, thrust_max]; the body rate takes an explicit Euler step of
// J domega/dt = tau - omega x J omega (X layout, torques from the new
// thrusts) and is clipped per axis; out = (collective thrust, body rate) for
// quad_step.
struct RotorState {
  float thr[4], w[3];
};

__device__ __forceinline__ void rotor_init(RotorState& r, const SolveDesc& d) {
#pragma unroll
  for (int i = 0; i < 4; ++i) r.thr[i] = d.thrust0[i];
#pragma unroll
  for (int i = 0; i < 3; ++i) r.w[i] = d.w0[i];
}

__device__ __forceinline__ void rotor_step(RotorState& r, const float udot[4], const SolveDesc& d, float out[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) r.thr[i] = fminf(fmaxf(fmaf(udot[i], d.dt, r.thr[i]), 0.0f), d.thrust_max);
  const float t1 = r.thr[0], t2 = r.thr[1], t3 = r.thr[2], t4 = r.thr[3];
  const float tau[3] = {d.rot_a * ((t1 - t2) + (t4 - t3)), d.rot_a * ((t2 - t1) + (t4 - t3)),
                        d.rot_kappa * ((t1 + t2) - (t3 + t4))};
  const float Jw[3] = {d.Jd[0] * r.w[0], d.Jd[1] * r.w[1], d.Jd[2] * r.w[2]};
  const float gyro[3] = {r.w[1] * Jw[2] - r.w[2] * Jw[1], r.w[2] * Jw[0] - r.w[0] * Jw[2],
                         r.w[0] * Jw[1] - r.w[1] * Jw[0]};
#pragma unroll
  for (int i = 0; i < 3; ++i)
    r.w[i] = fminf(fmaxf(fmaf(d.dt * d.Jinv[i], tau[i] - gyro[i], r.w[i]), -d.rate_max), d.rate_max);
  out[0] = (t1 + t2) + (t3 + t4);
  out[1] = r.w[0];
  out[2] = r.w[1];
  out[3] = r.w[2];
}

// One rollout step under the configured input: rs is used only for the
// rotor-thrust-rate input.
__device__ __forceinline__ void vehicle_step(RolloutState& s, RotorState& rs, const float u[4], const SolveDesc& d) {
  if (d.dyn == 1) {
    float uc[4];
    rotor_step(rs, u, d, uc);
    quad_step(s, uc, d.dt, d.inv_mass, d.gravity);
  } else {
    quad_step(s, u, d.dt, d.inv_mass, d.gravity);
  }
}

// 1 - cos(psi - psi_los) for the yaw psi of q and the bearing of (lx, ly)
// (eq. 6); atan2(0, 0) = 0 conventions for degenerate vectors.
__device__ __forceinline__ float alignment_term(const float q[4], float lx, float ly) {
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  float hx = 1.0f - 2.0f * (y * y + z * z), hy = 2.0f * (w * z + x * y);
  float hn = sqrtf(hx * hx + hy * hy);
  if (hn == 0.0f) { hx = 1.0f; hy = 0.0f; hn = 1.0f; }
  float ln = sqrtf(lx * lx + ly * ly);
  if (ln == 0.0f) { lx = 1.0f; ly = 0.0f; ln = 1.0f; }
  return 1.0f - (hx * lx + hy * ly) / (hn * ln);
}

// ---------------------------------------------------------------- positional encoding
// Feature f of PE(p), the encoded query point of the decoder's input
// (Section III-B): f < 3 the coordinates, then for k < F the blocks
// sin(2^k pi p) and cos(2^k pi p) over (x, y, z); 0 past the last feature.
// 2^k p is exact in float and sincospif reduces its argument exactly.
__device__ __forceinline__ float pe_feature(int f, float px, float py, float pz, int F) {
  if (f < 3) return f == 0 ? px : (f == 1 ? py : pz);
  const int j = f - 3;
  if (j >= 6 * F) return 0.0f;
  const int k = j / 6, r = j - 6 * k, c = r < 3 ? r : r - 3;
  const float v = ldexpf(c == 0 ? px : (c == 1 ? py : pz), k);
  float sn, cs;
  sincospif(v, &sn, &cs);
  return r < 3 ? sn : cs;
}

// ---------------------------------------------------------------- activations
// softplus(x) = log(1 + e^x) = max(x, 0) + log1p(e^-|x|): accurate form.
__device__ __forceinline__ float softplus_accurate(float x) {
  return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
}

// Analytic guidance field of eqs. 1-2 in gate-frame coordinates.
__device__ __forceinline__ float gate_sdf_analytic(float px, float py, float pz, float c,
                                                   float tan_a) {
  return c + fabsf(px) * tan_a - fmaxf(fabsf(py), fabsf(pz));
}

}  // namespace mppi
