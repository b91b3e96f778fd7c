// Per-solve descriptor shared by the host engine and the device kernels.
// It lives in device memory (one per in-flight solve); every pointer in it is
// a device address inside the engine's pool.
#pragma once
#include <stdint.h>

namespace mppi {

constexpr int kLatent = 64;
constexpr int kMaxG = 8;
constexpr int kMaxT = 128;
constexpr int kMaxK = 16384;

// Result block layout (doubles): U*[T][4], then these scalar slots.
enum ResultSlot : int {
  RES_U0 = 0,      // 4 doubles
  RES_JMIN = 4,
  RES_LOGETA = 5,
  RES_ESS = 6,
  RES_ETA = 7,
  RES_STATUS = 8,
  RES_TICK = 9,
  RES_SCALARS = 10
};

struct SolveDesc {
  // shape and identity
  int32_t K, T, G, flags;
  int32_t H, n_hidden, sdf_kind, U_len;  // U_len: entries of U_src (>= 1)
  uint64_t instance_id, seed;
  uint32_t tick_fixed;   // MPPI_TICK_RESIDENT -> read *tick_slot
  uint32_t q_off;        // 0: SDF at p_1..p_T, 1 -> index offset, see query_offset
  // dynamics (float32 copies of float64 inputs)
  float dt, inv_mass, gravity, pad0;
  float q0[4];
  // rotor-thrust-rate input (dyn == 1): X-layout lever a = arm / sqrt 2, yaw
  // drag per thrust, bounds, principal inertia and its inverse, the rotor
  // thrusts and body rate at x0
  int32_t dyn;
  float rot_a, rot_kappa, thrust_max, rate_max;
  float Jd[3], Jinv[3];
  float thrust0[4], w0[3];
  float L[16];           // lower-triangular noise factor, row-major
  float u_lo[4], u_hi[4];
  // costs
  float Q_gate, Q_vis, Q_sdf, d_safe, R_u;
  float fprog[3];        // v0 T dt + (p0 - wp): progress in the local frame
  float sdf_c, sdf_tan_alpha;
  double lambda, inv_lambda;
  double C0;             // Q_gate (|v0 T dt|^2 + 2 v0 T dt . (p0 - wp)): rollout-independent
  double hover[4];       // nominal of a new instance
  // inputs (device pointers into the request block / instance table)
  const double* U_src;   // U_len x 4 nominal or NULL -> hover
  const float* Rt;       // G x 9, R^T row-major
  const float* base;     // G x (T+1) x 3: R^T (p0 - t_g) + (t dt) R^T v0
  const float* z;        // G x 64 latent codes
  float* cfold;          // G x H: W1[:, 3:] z_g + b1, computed on the device in FP64
  float* cf_cache;       // instance's cached folded latents (G_max x H) or NULL
  uint32_t fold_cached;  // bit g: gate g not observed, take its fold from cf_cache
  uint32_t pad1;
  const float* los;      // T x 2: wp - p0 - v0 t dt (xy), for eq. 6
  double* U_resident;    // instance slot sequence (T_max x 4) or NULL
  uint32_t* tick_slot;   // instance slot tick
  // per-solve buffers (plain path)
  float* samples;        // [4][T][K]
  float* pos;            // [3][T+1][K] local-frame deviation positions
  float* sdf;            // [T][K] max-over-gates field at the query points
  float* Jpart;          // [K] progress + control + alignment
  float* J;              // [K] total cost minus C0
  double* wt;            // [K] unnormalised weights exp(-(J - rho) / lambda)
  double* wn;            // [K] normalised weights (optional, NULL when not asked)
  double* result;        // [4T + RES_SCALARS]
  // fused path
  double* partials;      // per tile: rho, eta, S[T][4]
  int32_t tile_rollouts; // rollouts per fused tile
  int32_t n_tiles;
  float* J_copy;         // [K] copy of J written with the normalised weights, or NULL
};

}  // namespace mppi
