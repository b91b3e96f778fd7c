// Fused path: one persistent launch per batch of solves.
//
// Each workgroup (8 waves) repeatedly takes a tile of R rollouts of some solve
// from a device work counter and runs the whole MPPI iteration on it
// (Section IV-A/B):
//   noise + clipping   all threads over (rollout, step) pairs -> LDS;
//   dynamics           one lane per rollout, serial over the horizon -> LDS
//                      positions, control / alignment / progress costs;
//   Gate-SDF decoder   32 query rows (rollout, step, gate) at a time; each wave
//                      owns H/8 neurons of every hidden layer and keeps their
//                      weights in VGPRs for the whole kernel; activations pass
//                      through LDS (ping-pong buffers) as matrix-core operands;
//                      the output dot and the max over gates end each chunk;
//   tile partial       FP64 (rho_i, eta_i, eta2_i, S_i[T][4]) of the tile;
//   merge              the workgroup that completes a solve's last tile
//                      combines the partials in tile-index order (so results
//                      do not depend on which workgroup ran which tile) and
//                      writes U*, the weights, the warm start and the tick.
//
// Precision variants of the hidden layers (FP32 accumulation throughout):
//   BF16    weights and activations rounded to bfloat16;
//   BF16X2  bfloat16 weights, activations split a = hi + lo (two products);
//   BF16X3  bfloat16 weights, a = hi + mid + lo (three products);
//   FP8     OCP E4M3 weights with a per-layer scale, E4M3 activations with a
//           static per-layer scale.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"
#include "weights.hpp"

namespace mppi {

using f32x4 = __attribute__((ext_vector_type(4))) float;
using bf16x8 = __attribute__((ext_vector_type(8))) __bf16;

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kRows = 32;     // query rows per chunk (two 16-row MFMA blocks)
constexpr int kTileR = 16;    // rollouts per tile
__host__ __device__ constexpr int kPartStride(int T) { return 4 + 4 * T; }

enum { P_BF16 = 1, P_BF16X2 = 2, P_FP8 = 3, P_BF16X3 = 4 };

template <int P> struct PrecTraits;
template <> struct PrecTraits<P_BF16> { static constexpr int splits = 1; static constexpr bool fp8 = false; };
template <> struct PrecTraits<P_BF16X2> { static constexpr int splits = 2; static constexpr bool fp8 = false; };
template <> struct PrecTraits<P_BF16X3> { static constexpr int splits = 3; static constexpr bool fp8 = false; };
template <> struct PrecTraits<P_FP8> { static constexpr int splits = 1; static constexpr bool fp8 = true; };

__device__ __forceinline__ uint16_t bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// softplus with the hardware base-2 exponential and logarithm:
// max(x, 0) + ln2 * log2(1 + 2^(-|x| log2 e)); absolute error ~1e-7.
__device__ __forceinline__ float softplus_fast(float x) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(x) * 1.4426950408889634f);
  return fmaf(__builtin_amdgcn_logf(1.0f + e), 0.6931471805599453f, fmaxf(x, 0.0f));
}

// LDS activation row stride in elements (bf16) / bytes (fp8): pad keeps
// 16-byte operand reads of 16 consecutive rows on distinct banks.
template <int H> __host__ __device__ constexpr int act_stride_bf16() { return H + 8; }
template <int H> __host__ __device__ constexpr int act_stride_fp8() { return H + 16; }

template <int P, int H>
__host__ __device__ constexpr size_t act_bytes() {
  return PrecTraits<P>::fp8 ? (size_t)2 * kRows * act_stride_fp8<H>()
                            : (size_t)2 * PrecTraits<P>::splits * kRows * act_stride_bf16<H>() * 2;
}

struct FusedLds {
  size_t act, w1p, hb, wo, cf, rt, base, los, samp, dp, hinge, pts, opart, jl, wt, fac, misc, total;
};

template <int P, int H>
__host__ __device__ FusedLds fused_lds(int Tm, int Gm, int max_tiles) {
  FusedLds L{};
  size_t o = 0;
  auto take = [&](size_t b) { const size_t r = o; o = (o + b + 15) / 16 * 16; return r; };
  L.act = take(act_bytes<P, H>());
  L.w1p = take(sizeof(float) * 4 * H);
  L.hb = take(sizeof(float) * 2 * H);      // hidden biases (up to 2 layers)
  L.wo = take(sizeof(float) * H);          // output row
  L.cf = take(sizeof(float) * Gm * H);
  L.rt = take(sizeof(float) * 9 * Gm);
  L.base = take(sizeof(float) * 3 * Gm * (Tm + 1));
  L.los = take(sizeof(float) * 2 * Tm);
  L.samp = take(sizeof(float) * 4 * kTileR * Tm);
  L.dp = take(sizeof(float) * 3 * kTileR * (Tm + 1));
  L.hinge = take(sizeof(float) * kTileR * Tm);
  L.pts = take(sizeof(float) * 4 * kRows);
  L.opart = take(sizeof(float) * kWaves * kRows);
  L.jl = take(sizeof(float) * 2 * kTileR);
  L.wt = take(sizeof(double) * (kTileR + 4));
  L.fac = take(sizeof(double) * max_tiles);
  L.misc = take(64);
  L.total = o;
  return L;
}

// Per-lane weight fragment of hidden layer l (A operand, 16x16x32): wave w,
// neuron block mb, K-step ks; lane holds W[m][32 ks + 8 (lane / 16) + j], j < 8,
// m = w H/8 + 16 mb + lane % 16.  BF16: 16 bytes; FP8: 8 bytes.
template <int H>
__host__ __device__ constexpr size_t frag_index(int l, int w, int mb, int ks, int lane) {
  return ((((size_t)l * kWaves + w) * (H / 8 / 16) + mb) * (H / 32) + ks) * 64 + lane;
}

template <int P, int H, int NHH>
__global__ __launch_bounds__(kThreads, 1) void k_fused(FusedBatch batch, DeviceWeights w, int Tm, int Gm,
                                                        int max_tiles) {
  using PT = PrecTraits<P>;
  constexpr int MW = H / kWaves;    // neurons per wave
  constexpr int MB = MW / 16;       // 16-neuron blocks per wave
  constexpr int KS = H / 32;        // K-steps of 32
  constexpr int NB = kRows / 16;    // 16-row blocks per chunk
  constexpr int NS = PT::splits;
  constexpr int STB = act_stride_bf16<H>();
  constexpr int ST8 = act_stride_fp8<H>();
  extern __shared__ __align__(16) char lds[];
  const FusedLds LL = fused_lds<P, H>(Tm, Gm, max_tiles);
  float* s_w1p = (float*)(lds + LL.w1p);
  float* s_hb = (float*)(lds + LL.hb);
  float* s_wo = (float*)(lds + LL.wo);
  float* s_cf = (float*)(lds + LL.cf);
  float* s_rt = (float*)(lds + LL.rt);
  float* s_base = (float*)(lds + LL.base);
  float* s_los = (float*)(lds + LL.los);
  float* s_samp = (float*)(lds + LL.samp);
  float* s_dp = (float*)(lds + LL.dp);
  float* s_hinge = (float*)(lds + LL.hinge);
  float* s_pts = (float*)(lds + LL.pts);
  float* s_opart = (float*)(lds + LL.opart);
  float* s_jl = (float*)(lds + LL.jl);
  double* s_wt = (double*)(lds + LL.wt);
  double* s_fac = (double*)(lds + LL.fac);
  int* s_misc = (int*)(lds + LL.misc);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 4, nl = lane & 15;

  // ---- weights of this wave's neurons, resident in VGPRs for the whole kernel
  using Frag = typename std::conditional<PT::fp8, long, bf16x8>::type;
  Frag wreg[NHH][MB][KS];
  float wsc[NHH];
#pragma unroll
  for (int l = 0; l < NHH; ++l) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const size_t fi = frag_index<H>(l, wave, mb, ks, lane);
        if constexpr (PT::fp8) wreg[l][mb][ks] = ((const long*)w.hidden_lp)[fi];
        else wreg[l][mb][ks] = __builtin_bit_cast(bf16x8, ((const uint4*)w.hidden_lp)[fi]);
      }
    }
    wsc[l] = PT::fp8 ? w.w_scale[l] * w.a_scale[l] : 1.0f;
  }
  for (int i = tid; i < 4 * H; i += kThreads) s_w1p[i] = w.w1p[i];
  for (int i = tid; i < NHH * H; i += kThreads) s_hb[i] = w.hbias[i];
  for (int i = tid; i < H; i += kThreads) s_wo[i] = w.wout[i];

  // Write this lane's 4 consecutive neurons (m0 .. m0+3) of row n to buffer buf.
  auto put_act = [&](int buf, int n, int m0, const float v[4], int layer_in) {
    if constexpr (PT::fp8) {
      // saturate to the largest E4M3 value: the conversion alone turns values
      // beyond the last rounding interval into NaN (activations are >= 0)
      const float inv = w.a_inv[layer_in];
      float q[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) q[i] = fminf(v[i] * inv, 448.0f);
      uint32_t word = __builtin_amdgcn_cvt_pk_fp8_f32(q[0], q[1], 0, false);
      word = __builtin_amdgcn_cvt_pk_fp8_f32(q[2], q[3], word, true);
      *(uint32_t*)(lds + LL.act + ((size_t)buf * kRows + n) * ST8 + m0) = word;
    } else {
      float r[4] = {v[0], v[1], v[2], v[3]};
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        uint16_t b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          b[i] = bf16_bits(r[i]);
          r[i] = r[i] - bf16_val(b[i]);
        }
        uint2 pk;
        pk.x = (uint32_t)b[0] | ((uint32_t)b[1] << 16);
        pk.y = (uint32_t)b[2] | ((uint32_t)b[3] << 16);
        *(uint2*)(lds + LL.act + (((size_t)(buf * NS + s) * kRows + n) * STB + m0) * 2) = pk;
      }
    }
  };

  while (true) {
    __syncthreads();
    if (tid == 0) s_misc[0] = (int)atomicAdd(batch.tile_counter, 1u);
    __syncthreads();
    const int tile = s_misc[0];
    if (tile >= batch.n_tiles) break;
    const int2 tl = batch.tiles[tile];
    const SolveDesc& d = batch.descs[tl.x];
    const int K = d.K, T = d.T, G = d.G;
    const int k0 = tl.y;
    const int Re = min(kTileR, K - k0);
    const uint32_t tick = d.tick_fixed == 0xFFFFFFFFu ? *d.tick_slot : d.tick_fixed;

    // ---- per-solve tables
    for (int i = tid; i < G * H; i += kThreads) s_cf[i] = d.cfold[i];
    for (int i = tid; i < 9 * G; i += kThreads) s_rt[i] = d.Rt[i];
    for (int i = tid; i < 3 * G * (T + 1); i += kThreads) s_base[i] = d.base[i];
    if (d.Q_vis != 0.0f)
      for (int i = tid; i < 2 * T; i += kThreads) s_los[i] = d.los[i];
    // ---- noise (Section IV-A): every (rollout, step) of the tile
    for (int i = tid; i < Re * T; i += kThreads) {
      const int kl = i / T, t = i - kl * T;
      float u[4];
      sample_control(d, (uint32_t)(k0 + kl), (uint32_t)t, tick, u);
      *(float4*)(s_samp + 4 * i) = make_float4(u[0], u[1], u[2], u[3]);
    }
    __syncthreads();
    // ---- dynamics: one lane per rollout
    if (tid < Re) {
      RolloutState s;
#pragma unroll
      for (int i = 0; i < 3; ++i) { s.dp[i] = 0.0f; s.dv[i] = 0.0f; }
#pragma unroll
      for (int i = 0; i < 4; ++i) s.q[i] = d.q0[i];
      float* dpk = s_dp + 3 * tid * (T + 1);
      dpk[0] = dpk[1] = dpk[2] = 0.0f;
      float Jc = 0.0f, Jv = 0.0f;
      for (int t = 0; t < T; ++t) {
        const float4 uu = *(const float4*)(s_samp + 4 * (tid * T + t));
        const float u[4] = {uu.x, uu.y, uu.z, uu.w};
        Jc = fmaf(u[0], u[0], fmaf(u[1], u[1], fmaf(u[2], u[2], fmaf(u[3], u[3], Jc))));
        if (d.Q_vis != 0.0f) Jv += alignment_term(s.q, s_los[2 * t] - s.dp[0], s_los[2 * t + 1] - s.dp[1]);
        quad_step(s, u, d.dt, d.inv_mass, d.gravity);
        dpk[3 * (t + 1) + 0] = s.dp[0];
        dpk[3 * (t + 1) + 1] = s.dp[1];
        dpk[3 * (t + 1) + 2] = s.dp[2];
      }
      const float Jg = s.dp[0] * s.dp[0] + s.dp[1] * s.dp[1] + s.dp[2] * s.dp[2] +
                       2.0f * (s.dp[0] * d.fprog[0] + s.dp[1] * d.fprog[1] + s.dp[2] * d.fprog[2]);
      s_jl[tid] = d.Q_gate * Jg + d.R_u * Jc + d.Q_vis * Jv;
    }
    // ---- Gate-SDF decoder over the tile's queries, kRows at a time
    const int Pc = kRows / G;                    // positions per chunk
    const int npos = Re * T;
    const int nchunks = (npos + Pc - 1) / Pc;
    for (int c = 0; c < nchunks; ++c) {
      __syncthreads();   // previous chunk done with s_pts / s_opart; dynamics done
      if (tid < kRows) {
        const int p = tid / G, g = tid - p * G;
        const int q = c * Pc + p;
        float px = 0.0f, py = 0.0f, pz = 0.0f;
        if (p < Pc && q < npos) {
          const int kl = q / T, t = q - kl * T;
          const int tp = t + (int)d.q_off;
          const float* dpp = s_dp + 3 * (kl * (T + 1) + tp);
          const float* R = s_rt + 9 * g;
          const float* b = s_base + 3 * (g * (T + 1) + tp);
          px = fmaf(R[0], dpp[0], fmaf(R[1], dpp[1], fmaf(R[2], dpp[2], b[0])));
          py = fmaf(R[3], dpp[0], fmaf(R[4], dpp[1], fmaf(R[5], dpp[2], b[1])));
          pz = fmaf(R[6], dpp[0], fmaf(R[7], dpp[1], fmaf(R[8], dpp[2], b[2])));
        }
        s_pts[4 * tid + 0] = px;
        s_pts[4 * tid + 1] = py;
        s_pts[4 * tid + 2] = pz;
        s_pts[4 * tid + 3] = (float)((p < Pc) ? g : 0);
      }
      __syncthreads();
      // layer 1 on the vector units, computed in the matrix-core output layout
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int m0 = wave * MW + 16 * mb + 4 * h;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int n = 16 * nb + nl;
          const float4 pt = *(const float4*)(s_pts + 4 * n);
          const int g = (int)pt.w;
          float v[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float4 wv = *(const float4*)(s_w1p + 4 * (m0 + i));
            const float x = fmaf(wv.x, pt.x, fmaf(wv.y, pt.y, fmaf(wv.z, pt.z, s_cf[g * H + m0 + i])));
            v[i] = softplus_fast(x);
          }
          put_act(0, n, m0, v, 0);
        }
      }
      // hidden H x H layers on the matrix cores
      float opart[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) opart[nb] = 0.0f;
#pragma unroll
      for (int l = 0; l < NHH; ++l) {
        __syncthreads();                 // layer input complete in buffer (l & 1)
        const int src = l & 1;
        f32x4 acc[MB][NB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            if constexpr (PT::fp8) acc[mb][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            else acc[mb][nb] = *(const f32x4*)(s_hb + l * H + wave * MW + 16 * mb + 4 * h);
          }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          if constexpr (PT::fp8) {
            long bfr[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              bfr[nb] = *(const long*)(lds + LL.act + ((size_t)src * kRows + 16 * nb + nl) * ST8 + 32 * ks + 8 * h);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(wreg[l][mb][ks], bfr[nb], acc[mb][nb], 0, 0, 0);
          } else {
            bf16x8 bfr[NS][NB];
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
                bfr[s][nb] = __builtin_bit_cast(
                    bf16x8, *(const uint4*)(lds + LL.act +
                                            (((size_t)(src * NS + s) * kRows + 16 * nb + nl) * STB + 32 * ks + 8 * h) * 2));
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
              for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                  acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wreg[l][mb][ks], bfr[s][nb], acc[mb][nb], 0, 0, 0);
          }
        }
        // epilogue: bias (FP8 scale), softplus; next layer's operand or output dot
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const int m0 = wave * MW + 16 * mb + 4 * h;
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float x = PT::fp8 ? fmaf(acc[mb][nb][i], wsc[l], s_hb[l * H + m0 + i]) : acc[mb][nb][i];
              v[i] = softplus_fast(x);
            }
            if (l + 1 < NHH) {
              put_act(src ^ 1, 16 * nb + nl, m0, v, l + 1);
            } else {
#pragma unroll
              for (int i = 0; i < 4; ++i) opart[nb] = fmaf(s_wo[m0 + i], v[i], opart[nb]);
            }
          }
        }
      }
      // output layer: reduce the lane groups holding the same row, then the waves
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        float v = opart[nb];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (h == 0) s_opart[wave * kRows + 16 * nb + nl] = v;
      }
      __syncthreads();
      if (tid < kRows) {
        float sv = w.bout;
        float acc0 = 0.0f;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) acc0 += s_opart[ww * kRows + tid];
        sv += acc0;
        // max over the gates of each position (rows p G .. p G + G - 1)
        const int p = tid / G;
        float best = sv;
        for (int g = 1; g < G; ++g) {
          const float o = __shfl(sv, p * G + g, 64);
          if (p * G + g < kRows) best = fmaxf(best, o);
        }
        const int q = c * Pc + p;
        if (tid == p * G && p < Pc && q < npos) s_hinge[q] = fmaxf(0.0f, d.d_safe - best);
      }
    }
    __syncthreads();
    // ---- per-rollout costs and the tile's FP64 partials
    if (tid < Re) {
      float hs = 0.0f;
      for (int t = 0; t < T; ++t) hs += s_hinge[tid * T + t];
      const float J = s_jl[tid] + d.Q_sdf * hs;
      s_jl[kTileR + tid] = J;
      d.J[k0 + tid] = J;
    }
    __syncthreads();
    if (tid == 0) {
      double rho = INFINITY;
      for (int k = 0; k < Re; ++k) {
        const float J = s_jl[kTileR + k];
        if (isfinite(J)) rho = fmin(rho, (double)J);
      }
      double eta = 0.0, eta2 = 0.0;
      for (int k = 0; k < Re; ++k) {
        const float J = s_jl[kTileR + k];
        const double wt = (isfinite(J) && isfinite(rho)) ? exp(-((double)J - rho) * d.inv_lambda) : 0.0;
        s_wt[k] = wt;
        eta += wt;
        eta2 += wt * wt;
      }
      s_wt[kTileR] = rho;
      s_wt[kTileR + 1] = eta;
      s_wt[kTileR + 2] = eta2;
    }
    __syncthreads();
    const int ti = k0 / d.tile_rollouts;
    double* part = d.partials + (size_t)ti * kPartStride(T);
    if (tid < 3) part[tid] = s_wt[kTileR + tid];
    for (int i = tid; i < 4 * T; i += kThreads) {
      double sacc = 0.0;
      for (int k = 0; k < Re; ++k) sacc = fma(s_wt[k], (double)s_samp[4 * (k * T) + i], sacc);
      part[4 + i] = sacc;
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      const uint32_t prev = atomicAdd(d.tiles_done, 1u);
      s_misc[1] = (prev + 1 == (uint32_t)d.n_tiles) ? 1 : 0;
    }
    __syncthreads();
    if (!s_misc[1]) continue;
    // ---- last tile of this solve: merge the partials in tile order
    __threadfence();
    if (tid == 0) {
      double rho = INFINITY;
      for (int i = 0; i < d.n_tiles; ++i) {
        const double* pi = d.partials + (size_t)i * kPartStride(T);
        if (pi[1] > 0.0) rho = fmin(rho, pi[0]);
      }
      double eta = 0.0, eta2 = 0.0;
      for (int i = 0; i < d.n_tiles; ++i) {
        const double* pi = d.partials + (size_t)i * kPartStride(T);
        if (pi[1] > 0.0) {
          const double f = exp(-(pi[0] - rho) * d.inv_lambda);
          eta = fma(pi[1], f, eta);
          eta2 = fma(pi[2], f * f, eta2);
        }
      }
      s_wt[0] = rho;
      s_wt[1] = eta;
      s_wt[2] = eta2;
      *d.tiles_done = 0u;
    }
    __syncthreads();
    for (int j = tid; j < d.n_tiles; j += kThreads) {
      const double* pj = d.partials + (size_t)j * kPartStride(T);
      s_fac[j] = (pj[1] > 0.0 && isfinite(s_wt[0])) ? exp(-(pj[0] - s_wt[0]) * d.inv_lambda) : 0.0;
    }
    __syncthreads();
    const double rho = s_wt[0], eta = s_wt[1], eta2 = s_wt[2];
    const bool ok = isfinite(rho) && eta > 0.0;
    double* res = d.result;
    for (int i = tid; i < 4 * T; i += kThreads) {
      const int t = i >> 2, ch = i & 3;
      double U;
      if (ok) {
        double sacc = 0.0;
        for (int j = 0; j < d.n_tiles; ++j)
          sacc = fma(d.partials[(size_t)j * kPartStride(T) + 4 + i], s_fac[j], sacc);
        U = sacc / eta;
      } else {
        const int tt = t < d.U_len ? t : d.U_len - 1;
        U = d.U_src ? d.U_src[tt * 4 + ch] : d.hover[ch];
      }
      res[i] = U;
      if (t == 0) res[4 * T + RES_U0 + ch] = U;
      if (ok && d.U_resident && !(d.flags & 1)) {
        if (t >= 1) d.U_resident[(t - 1) * 4 + ch] = U;
        if (t == T - 1) d.U_resident[t * 4 + ch] = U;
      }
    }
    if (d.wn)
      for (int k = tid; k < K; k += kThreads) {
        const float J = d.J[k];
        d.wn[k] = (ok && isfinite(J)) ? exp(-((double)J - rho) * d.inv_lambda) / eta : 0.0;
      }
    if (tid == 0) {
      double* r = res + 4 * T;
      r[RES_TICK] = (double)tick;
      if (ok) {
        const double jmin = rho + d.C0;
        r[RES_STATUS] = 0.0;
        r[RES_JMIN] = jmin;
        r[RES_LOGETA] = log(eta) - jmin * d.inv_lambda;
        r[RES_ESS] = eta * eta / eta2;
        r[RES_ETA] = eta;
      } else {
        r[RES_STATUS] = -5.0;
        r[RES_JMIN] = NAN;
        r[RES_LOGETA] = NAN;
        r[RES_ESS] = 0.0;
        r[RES_ETA] = 0.0;
      }
      if (d.tick_slot) *d.tick_slot = tick + 1u;
    }
  }
}

// Zero the batch's work counter and every solve's tile counter.
__global__ void k_fused_prep(FusedBatch b, int n_solves) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *b.tile_counter = 0u;
  if (i < n_solves) *b.descs[i].tiles_done = 0u;
}

// ------------------------------------------------------------------ host side

template <int P, int H, int NHH>
static hipError_t launch_fused_t(const FusedBatch& b, const DeviceWeights& w, int Tm, int Gm,
                                 int max_tiles, hipStream_t s) {
  const FusedLds L = fused_lds<P, H>(Tm, Gm, max_tiles);
  static int max_set = 0;
  if ((int)L.total > max_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_fused<P, H, NHH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
    if (e != hipSuccess) return e;
    max_set = (int)L.total;
  }
  int dev = 0, ncu = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int grid = std::max(1, std::min(b.n_tiles, ncu));
  hipLaunchKernelGGL((k_fused<P, H, NHH>), dim3(grid), dim3(kThreads), L.total, s, b, w, Tm, Gm, max_tiles);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_fused_p(const FusedBatch& b, const DeviceWeights& w, int Tm, int Gm, int mt,
                                 hipStream_t s) {
  const int nhh = w.n_hidden - 1;
  if (w.H == 128 && nhh == 1) return launch_fused_t<P, 128, 1>(b, w, Tm, Gm, mt, s);
  if (w.H == 128 && nhh == 2) return launch_fused_t<P, 128, 2>(b, w, Tm, Gm, mt, s);
  if (w.H == 256 && nhh == 1) return launch_fused_t<P, 256, 1>(b, w, Tm, Gm, mt, s);
  if (w.H == 256 && nhh == 2) return launch_fused_t<P, 256, 2>(b, w, Tm, Gm, mt, s);
  return hipErrorInvalidValue;
}

hipError_t launch_fused(const FusedBatch& b, int n_solves, const DeviceWeights& w, int max_T, int max_G,
                        int max_tiles, hipStream_t s, hipEvent_t begin, hipEvent_t end) {
  hipLaunchKernelGGL(k_fused_prep, dim3((n_solves + 255) / 256), dim3(256), 0, s, b, n_solves);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (begin) hipEventRecord(begin, s);
  switch (w.precision) {
    case P_BF16: e = launch_fused_p<P_BF16>(b, w, max_T, max_G, max_tiles, s); break;
    case P_BF16X2: e = launch_fused_p<P_BF16X2>(b, w, max_T, max_G, max_tiles, s); break;
    case P_BF16X3: e = launch_fused_p<P_BF16X3>(b, w, max_T, max_G, max_tiles, s); break;
    case P_FP8: e = launch_fused_p<P_FP8>(b, w, max_T, max_G, max_tiles, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (end) hipEventRecord(end, s);
  return hipSuccess;
}

int fused_tile_rollouts(int, int, int) { return kTileR; }

bool fused_supported(int precision, int H, int n_hidden) {
  if (!(precision == P_BF16 || precision == P_BF16X2 || precision == P_BF16X3 || precision == P_FP8)) return false;
  return (H == 128 || H == 256) && (n_hidden == 2 || n_hidden == 3);
}

size_t fused_lds_bytes(int precision, int H, int Tm, int Gm, int max_tiles) {
  auto pick = [&](auto p_tag) -> size_t {
    constexpr int P = decltype(p_tag)::value;
    return H == 128 ? fused_lds<P, 128>(Tm, Gm, max_tiles).total : fused_lds<P, 256>(Tm, Gm, max_tiles).total;
  };
  switch (precision) {
    case P_BF16: return pick(std::integral_constant<int, P_BF16>{});
    case P_BF16X2: return pick(std::integral_constant<int, P_BF16X2>{});
    case P_BF16X3: return pick(std::integral_constant<int, P_BF16X3>{});
    case P_FP8: return pick(std::integral_constant<int, P_FP8>{});
  }
  return 0;
}

// ---- weight packing -------------------------------------------------------

static uint16_t host_bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// OCP E4M3 (bias 7, max 448, no infinities), round to nearest even, saturating.
static uint8_t host_e4m3(float x) {
  const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
  float a = fabsf(x);
  if (!(a == a)) return 0x7F;
  if (a >= 448.0f) return sign | 0x7E;
  int e;
  const double m = frexp((double)a, &e);   // a = m 2^e, m in [0.5, 1)
  double q;
  if (a < 0.015625f) q = nearbyint((double)a * 512.0) / 512.0;  // subnormal grid 2^-9
  else q = ldexp(nearbyint(m * 16.0), e - 4);
  if (q >= 448.0) return sign | 0x7E;
  if (q == 0.0) return sign;
  int qe;
  const double qm = frexp(q, &qe);
  if (q < 0.015625) return sign | (uint8_t)nearbyint(q * 512.0);   // exponent field 0
  const int E = qe - 1 + 7;                                        // q = 1.f 2^(qe-1)
  const int F = (int)nearbyint((qm * 2.0 - 1.0) * 8.0);
  return sign | (uint8_t)((E << 3) | F);
}

int pack_lowp_weights(int precision, int H, int n_hidden, const mppi_sdf_weights* w,
                      std::vector<uint8_t>& blob, std::vector<float>& w_scale,
                      std::vector<float>& a_scale, std::vector<float>& a_inv) {
  if (!fused_supported(precision, H, n_hidden)) return MPPI_EINVAL;
  const int nhh = n_hidden - 1;
  const int MB = H / kWaves / 16, KS = H / 32;
  const bool fp8 = precision == P_FP8;
  const size_t esz = fp8 ? 8 : 16;
  blob.assign((size_t)nhh * kWaves * MB * KS * 64 * esz, 0);
  w_scale.assign(nhh, 1.0f);
  a_scale.assign(nhh, 1.0f);
  a_inv.assign(nhh, 1.0f);
  for (int l = 0; l < nhh; ++l) {
    const float* W = w->W[l + 1];
    float scale = 1.0f;
    if (fp8) {
      float amax = 0.0f;
      for (size_t i = 0; i < (size_t)H * H; ++i) amax = std::max(amax, fabsf(W[i]));
      scale = amax > 0.0f ? amax / 448.0f : 1.0f;
      w_scale[l] = scale;
      const float as = w->act_scale[l];
      if (!(as > 0.0f) || !std::isfinite(as)) return MPPI_EINVAL;
      a_scale[l] = as;
      a_inv[l] = 1.0f / as;
    }
    for (int wv = 0; wv < kWaves; ++wv)
      for (int mb = 0; mb < MB; ++mb)
        for (int ks = 0; ks < KS; ++ks)
          for (int lane = 0; lane < 64; ++lane) {
            const int m = wv * (H / kWaves) + 16 * mb + lane % 16;
            const size_t fi = ((((size_t)l * kWaves + wv) * MB + mb) * KS + ks) * 64 + lane;
            for (int j = 0; j < 8; ++j) {
              const int k = 32 * ks + 8 * (lane / 16) + j;
              const float v = W[(size_t)m * H + k];
              if (fp8) {
                blob[fi * 8 + j] = host_e4m3(v / scale);
              } else {
                const uint16_t b = host_bf16_rne(v);
                memcpy(&blob[fi * 16 + 2 * j], &b, 2);
              }
            }
          }
  }
  return MPPI_OK;
}

}  // namespace mppi
