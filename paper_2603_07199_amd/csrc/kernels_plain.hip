// Plain path: one solve per launch sequence.
//   k_rollout   one lane per rollout: noise, clipping, dynamics, progress,
//               control and alignment costs (Section IV-A/B, eqs. 5, 6, 9);
//   k_sdf_f32   Gate-SDF decoder over every (step, rollout, gate) query on
//               FP32 matrix cores, max over gates (Section III-B, IV-B-3);
//   k_sdf_analytic  the guidance field of eqs. 1-2 instead of the decoder;
//   k_cost      per-rollout SDF hinge sum (eqs. 7-8) added to the rest (eq. 9);
//   k_lse       FP64 minimum, unnormalised weights and their sum (eq. mppi_update);
//   k_wavg      FP64 weighted average of the sampled controls, warm start.
// Reductions use fixed-order trees, so a solve is bitwise reproducible.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>

#include <mutex>

#include "device_common.hpp"
#include "kernels.hpp"
#include "weights.hpp"

namespace mppi {

using f32x4 = __attribute__((ext_vector_type(4))) float;

__device__ __forceinline__ uint32_t solve_tick(const SolveDesc& d) {
  return d.tick_fixed == 0xFFFFFFFFu ? *d.tick_slot : d.tick_fixed;
}

// ------------------------------------------------------------------ latent fold
__global__ __launch_bounds__(256) void k_fold(const SolveDesc* __restrict__ descs, DeviceWeights w) {
  fold_gate(descs[blockIdx.y], blockIdx.x, w);
}

hipError_t launch_fold(const SolveDesc* descs, int n_solves, int G_max, const DeviceWeights& w,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_fold, dim3(G_max, n_solves), dim3(256), 0, s, descs, w);
  return hipGetLastError();
}

// ------------------------------------------------------------------ rollout
__global__ __launch_bounds__(256) void k_rollout(const SolveDesc* __restrict__ dd) {
  const SolveDesc& d = *dd;
  const int K = d.K, T = d.T;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t tick = solve_tick(d);
  if (k == 0) d.result[4 * T + RES_TICK] = (double)tick;
  if (k >= K) return;
  RolloutState s;
#pragma unroll
  for (int i = 0; i < 3; ++i) { s.dp[i] = 0.0f; s.dv[i] = 0.0f; }
#pragma unroll
  for (int i = 0; i < 4; ++i) s.q[i] = d.q0[i];
  RotorState rs;
  rotor_init(rs, d);
  const size_t TK = (size_t)T * K, T1K = (size_t)(T + 1) * K;
  for (int c = 0; c < 3; ++c) d.pos[c * T1K + k] = 0.0f;
  float Jc = 0.0f, Jv = 0.0f;
  for (int t = 0; t < T; ++t) {
    float u[4];
    sample_control(d, (uint32_t)k, (uint32_t)t, tick, u);
#pragma unroll
    for (int c = 0; c < 4; ++c) d.samples[c * TK + (size_t)t * K + k] = u[c];
    Jc = fmaf(u[0], u[0], fmaf(u[1], u[1], fmaf(u[2], u[2], fmaf(u[3], u[3], Jc))));
    if (d.Q_vis != 0.0f)
      Jv += alignment_term(s.q, d.los[2 * t] - s.dp[0], d.los[2 * t + 1] - s.dp[1]);
    vehicle_step(s, rs, u, d);
#pragma unroll
    for (int c = 0; c < 3; ++c) d.pos[c * T1K + (size_t)(t + 1) * K + k] = s.dp[c];
  }
  // progress (eq. 5, telescoped) in the local frame; the constant part is d.C0
  const float Jg = s.dp[0] * s.dp[0] + s.dp[1] * s.dp[1] + s.dp[2] * s.dp[2] +
                   2.0f * (s.dp[0] * d.fprog[0] + s.dp[1] * d.fprog[1] + s.dp[2] * d.fprog[2]);
  d.Jpart[k] = d.Q_gate * Jg + d.R_u * Jc + d.Q_vis * Jv;
}

// ------------------------------------------------------------------ SDF, FP32 MFMA
// Block of 256 threads (4 waves) owns 64 query rows; a row is one (step,
// rollout, gate) query, gates fastest, P = 64 / G positions per block.
// Activations live transposed in LDS (actT[k][row]); hidden-layer weights
// stream from L2 as pre-packed 16x16x4 operand fragments.  Each wave owns
// H/64 blocks of 16 output neurons for all 64 rows.
template <int H, bool PE>
__global__ __launch_bounds__(256) void k_sdf_f32(const SolveDesc* __restrict__ dd, DeviceWeights w) {
  const SolveDesc& d = *dd;
  constexpr int ST = H <= 256 ? 80 : 68;  // row stride of actT (floats)
  constexpr int MBW = H / 64;             // 16-neuron blocks per wave
  extern __shared__ float smem[];
  float* actT = smem;                     // H x ST
  float* pts = actT + H * ST;             // 64 x 3
  float* part = pts + 192;                // 4 x 64
  float* featT = part + 256;              // positional encoding: 4 feat_ksteps x ST, featT[f][row]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int G = d.G, K = d.K, T = d.T;
  const int P = 64 / G;
  const long npos = (long)K * T;
  const long pos0 = (long)blockIdx.x * P;

  if (tid < 64) {
    const int p = tid / G, g = tid - p * G;
    const long idx = pos0 + p;
    float px = 0.0f, py = 0.0f, pz = 0.0f;
    if (p < P && idx < npos) {
      const int t = (int)(idx / K), k = (int)(idx - (long)t * K);
      const int tp = t + (int)d.q_off;
      const size_t T1K = (size_t)(T + 1) * K;
      const float x = d.pos[(size_t)tp * K + k], y = d.pos[T1K + (size_t)tp * K + k],
                  z = d.pos[2 * T1K + (size_t)tp * K + k];
      const float* R = d.Rt + 9 * g;
      const float* b = d.base + ((size_t)g * (T + 1) + tp) * 3;
      px = fmaf(R[0], x, fmaf(R[1], y, fmaf(R[2], z, b[0])));
      py = fmaf(R[3], x, fmaf(R[4], y, fmaf(R[5], z, b[1])));
      pz = fmaf(R[6], x, fmaf(R[7], y, fmaf(R[8], z, b[2])));
    }
    pts[tid * 3 + 0] = px;
    pts[tid * 3 + 1] = py;
    pts[tid * 3 + 2] = pz;
  }
  __syncthreads();

  const int h = lane >> 4, nl = lane & 15;
  if constexpr (!PE) {
    // layer 1 on the vector units: softplus(W1[:, :3] p + c_g)
    for (int e = tid; e < H * 64; e += 256) {
      const int n = e & 63, m = e >> 6;
      const int g = (n / G < P) ? n % G : 0;
      const float x = fmaf(w.w1p[m * 4 + 0], pts[n * 3 + 0],
                           fmaf(w.w1p[m * 4 + 1], pts[n * 3 + 1],
                                fmaf(w.w1p[m * 4 + 2], pts[n * 3 + 2], d.cfold[g * H + m])));
      actT[m * ST + n] = softplus_accurate(x);
    }
  } else {
    // encoded point: the features of the 64 rows, then layer 1 on the matrix
    // cores, softplus(W1[:, :n_feat] PE(p) + c_g), K-steps of 4 features
    const int KQ = w.feat_ksteps;
    for (int e = tid; e < 4 * KQ * 64; e += 256) {
      const int n = e & 63, f = e >> 6;
      featT[f * ST + n] = pe_feature(f, pts[n * 3 + 0], pts[n * 3 + 1], pts[n * 3 + 2], w.pe_freqs);
    }
    __syncthreads();
    f32x4 acc[MBW][4];
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb) {
      const int m0 = 16 * (wave * MBW + mb) + 4 * h;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int n = 16 * nb + nl;
        const int g = (n / G < P) ? n % G : 0;
        const float* c = d.cfold + g * H + m0;
        acc[mb][nb] = f32x4{c[0], c[1], c[2], c[3]};
      }
    }
    for (int ks = 0; ks < KQ; ++ks) {
      float bf[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) bf[nb] = featT[(4 * ks + h) * ST + 16 * nb + nl];
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb) {
        const float a = w.w1pe[((size_t)(wave * MBW + mb) * KQ + ks) * 64 + lane];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bf[nb], acc[mb][nb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb) {
      const int m0 = 16 * (wave * MBW + mb) + 4 * h;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          actT[(m0 + i) * ST + 16 * nb + nl] = softplus_accurate(acc[mb][nb][i]);
    }
  }
  __syncthreads();

  for (int l = 0; l < d.n_hidden - 1; ++l) {
    const float* Wp = w.hidden_f32 + (size_t)l * H * H;
    const float* bias = w.hbias + l * H;
    f32x4 acc[MBW][4];
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb) {
      const int m0 = 16 * (wave * MBW + mb) + 4 * h;
      const f32x4 bv = {bias[m0], bias[m0 + 1], bias[m0 + 2], bias[m0 + 3]};
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = bv;
    }
#pragma unroll 4
    for (int ks = 0; ks < H / 4; ++ks) {
      float bf[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) bf[nb] = actT[(4 * ks + h) * ST + 16 * nb + nl];
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb) {
        const float a = Wp[((size_t)(wave * MBW + mb) * (H / 4) + ks) * 64 + lane];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bf[nb], acc[mb][nb], 0, 0, 0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb) {
      const int m0 = 16 * (wave * MBW + mb) + 4 * h;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          actT[(m0 + i) * ST + 16 * nb + nl] = softplus_accurate(acc[mb][nb][i]);
    }
    __syncthreads();
  }

  {  // output layer: partial dot products over m = part (mod 4)
    const int n = tid & 63, q = tid >> 6;
    float s = 0.0f;
    for (int m = q; m < H; m += 4) s = fmaf(w.wout[m], actT[m * ST + n], s);
    part[q * 64 + n] = s;
  }
  __syncthreads();
  if (tid < P) {
    const long idx = pos0 + tid;
    if (idx < npos) {
      float best = -INFINITY;
      for (int g = 0; g < G; ++g) {
        const int r = tid * G + g;
        const float s = ((part[r] + part[64 + r]) + (part[128 + r] + part[192 + r])) + w.bout;
        best = fmaxf(best, s);
      }
      d.sdf[idx] = best;
    }
  }
}

// ------------------------------------------------------------------ analytic SDF
__global__ __launch_bounds__(256) void k_sdf_analytic(const SolveDesc* __restrict__ dd) {
  const SolveDesc& d = *dd;
  const int K = d.K, T = d.T;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)K * T) return;
  const int t = (int)(idx / K), k = (int)(idx - (long)t * K);
  const int tp = t + (int)d.q_off;
  const size_t T1K = (size_t)(T + 1) * K;
  const float x = d.pos[(size_t)tp * K + k], y = d.pos[T1K + (size_t)tp * K + k],
              z = d.pos[2 * T1K + (size_t)tp * K + k];
  float best = -INFINITY;
  for (int g = 0; g < d.G; ++g) {
    const float* R = d.Rt + 9 * g;
    const float* b = d.base + ((size_t)g * (T + 1) + tp) * 3;
    const float px = fmaf(R[0], x, fmaf(R[1], y, fmaf(R[2], z, b[0])));
    const float py = fmaf(R[3], x, fmaf(R[4], y, fmaf(R[5], z, b[1])));
    const float pz = fmaf(R[6], x, fmaf(R[7], y, fmaf(R[8], z, b[2])));
    best = fmaxf(best, gate_sdf_analytic(px, py, pz, d.sdf_c, d.sdf_tan_alpha));
  }
  d.sdf[idx] = best;
}

// ------------------------------------------------------------------ costs
__global__ __launch_bounds__(256) void k_cost(const SolveDesc* __restrict__ dd) {
  const SolveDesc& d = *dd;
  const int K = d.K, T = d.T;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  float hs = 0.0f;
  for (int t = 0; t < T; ++t) hs += fmaxf(0.0f, d.d_safe - d.sdf[(size_t)t * K + k]);
  d.J[k] = d.Jpart[k] + d.Q_sdf * hs;
}

// ------------------------------------------------------------------ FP64 reductions
constexpr int kRedThreads = 1024;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = sh[tid] + sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_min(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = fmin(sh[tid], sh[tid + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// rho = min J, wt = exp(-(J - rho) / lambda), eta = sum wt (non-finite J -> 0).
__global__ __launch_bounds__(kRedThreads) void k_lse(const SolveDesc* __restrict__ dd) {
  __shared__ double sh[kRedThreads];
  const SolveDesc& d = *dd;
  const int K = d.K, T = d.T, tid = threadIdx.x;
  double mn = INFINITY;
  for (int k = tid; k < K; k += kRedThreads) {
    const float j = d.J[k];
    if (isfinite(j)) mn = fmin(mn, (double)j);
  }
  const double rho = block_min(mn, sh);
  double e = 0.0, e2 = 0.0;
  for (int k = tid; k < K; k += kRedThreads) {
    const float j = d.J[k];
    const double wt = (isfinite(j) && isfinite(rho)) ? exp(-((double)j - rho) * d.inv_lambda) : 0.0;
    d.wt[k] = wt;
    e += wt;
    e2 += wt * wt;
  }
  const double eta = block_sum(e, sh);
  const double eta2 = block_sum(e2, sh);
  if (tid == 0) {
    double* r = d.result + 4 * T;
    if (!isfinite(rho) || !(eta > 0.0)) {
      r[RES_STATUS] = -5.0;  // every cost non-finite
      r[RES_JMIN] = NAN;
      r[RES_LOGETA] = NAN;
      r[RES_ESS] = 0.0;
      r[RES_ETA] = 0.0;
    } else {
      const double jmin = rho + d.C0;
      r[RES_STATUS] = 0.0;
      r[RES_JMIN] = jmin;
      r[RES_LOGETA] = log(eta) - jmin * d.inv_lambda;
      r[RES_ESS] = eta * eta / eta2;
      r[RES_ETA] = eta;
    }
  }
}

// U*_t = sum_k wt_k u_k,t / eta; one block per step t.  Writes the shifted
// sequence into the instance slot (warm start) and advances the tick.
__global__ __launch_bounds__(256) void k_wavg(const SolveDesc* __restrict__ dd) {
  __shared__ double sh[256];
  const SolveDesc& d = *dd;
  const int K = d.K, T = d.T, t = blockIdx.x, tid = threadIdx.x;
  const double* r = d.result + 4 * T;
  const bool ok = r[RES_STATUS] == 0.0;
  const double eta = r[RES_ETA];
  double U[4];
  if (ok) {
    const size_t TK = (size_t)T * K;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = tid; k < K; k += 256) {
      const double wt = d.wt[k];
#pragma unroll
      for (int c = 0; c < 4; ++c) s[c] = fma(wt, (double)d.samples[c * TK + (size_t)t * K + k], s[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) U[c] = block_sum(s[c], sh) / eta;
  } else {
    const int ti = t < d.U_len ? t : d.U_len - 1;
#pragma unroll
    for (int c = 0; c < 4; ++c) U[c] = d.U_src ? d.U_src[ti * 4 + c] : d.hover[c];
  }
  if (tid == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      d.result[t * 4 + c] = U[c];
      if (t == 0) d.result[4 * T + RES_U0 + c] = U[c];
    }
    if (ok && d.U_resident && !(d.flags & 1)) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (t >= 1) d.U_resident[(t - 1) * 4 + c] = U[c];
        if (t == T - 1) d.U_resident[t * 4 + c] = U[c];
      }
    }
    if (t == 0 && d.tick_slot) *d.tick_slot = (uint32_t)r[RES_TICK] + 1u;
  }
  if (t == 0 && d.wn) {
    for (int k = tid; k < K; k += 256) d.wn[k] = ok ? d.wt[k] / eta : 0.0;
  }
}

// ------------------------------------------------------------------ launchers
template <int H, bool PE>
static hipError_t launch_sdf_f32_h(const SolveDesc* dd, const DeviceWeights& w, long npos, int G,
                                   hipStream_t s) {
  constexpr int ST = H <= 256 ? 80 : 68;
  const size_t lds = ((size_t)H * ST + 192 + 256 + (size_t)4 * w.feat_ksteps * ST) * sizeof(float);
  {
    // raise the kernel's dynamic LDS limit to the largest size launched so far
    static std::mutex mu;
    static size_t max_set = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (lds > max_set) {
      hipError_t e = hipFuncSetAttribute((const void*)k_sdf_f32<H, PE>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      max_set = lds;
    }
  }
  const int P = 64 / G;
  const long blocks = (npos + P - 1) / P;
  hipLaunchKernelGGL((k_sdf_f32<H, PE>), dim3((unsigned)blocks), dim3(256), lds, s, dd, w);
  return hipGetLastError();
}

hipError_t launch_plain(const SolveDesc* dd, const PlainShape& sh, const DeviceWeights& w,
                        hipStream_t s, hipEvent_t sdf_begin, hipEvent_t sdf_end) {
  const int K = sh.K, T = sh.T;
  hipError_t e = hipSuccess;
  if (sh.sdf_kind == 0) {
    e = launch_fold(dd, 1, sh.G, w, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_rollout, dim3((K + 255) / 256), dim3(256), 0, s, dd);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (sdf_begin) hipEventRecord(sdf_begin, s);
  const long npos = (long)K * T;
  if (sh.sdf_kind == 1) {
    hipLaunchKernelGGL(k_sdf_analytic, dim3((unsigned)((npos + 255) / 256)), dim3(256), 0, s, dd);
    e = hipGetLastError();
  } else {
    const bool pe = w.feat_ksteps > 0;
    switch (w.H) {
      case 64: e = pe ? launch_sdf_f32_h<64, true>(dd, w, npos, sh.G, s) : launch_sdf_f32_h<64, false>(dd, w, npos, sh.G, s); break;
      case 128: e = pe ? launch_sdf_f32_h<128, true>(dd, w, npos, sh.G, s) : launch_sdf_f32_h<128, false>(dd, w, npos, sh.G, s); break;
      case 256: e = pe ? launch_sdf_f32_h<256, true>(dd, w, npos, sh.G, s) : launch_sdf_f32_h<256, false>(dd, w, npos, sh.G, s); break;
      case 512: e = pe ? launch_sdf_f32_h<512, true>(dd, w, npos, sh.G, s) : launch_sdf_f32_h<512, false>(dd, w, npos, sh.G, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  if (sdf_end) hipEventRecord(sdf_end, s);
  hipLaunchKernelGGL(k_cost, dim3((K + 255) / 256), dim3(256), 0, s, dd);
  hipLaunchKernelGGL(k_lse, dim3(1), dim3(kRedThreads), 0, s, dd);
  hipLaunchKernelGGL(k_wavg, dim3(T), dim3(256), 0, s, dd);
  return hipGetLastError();
}

}  // namespace mppi
