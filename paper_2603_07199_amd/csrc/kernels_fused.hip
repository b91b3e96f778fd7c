// Fused path: one persistent launch per batch of solves.
//
// Each workgroup repeatedly takes a tile of 16 rollouts of some solve from a
// device work counter and runs the whole MPPI iteration on it (Section IV-A/B):
//   noise + clipping   all threads over (rollout, step) pairs -> LDS;
//   dynamics           one lane per rollout, serial over the horizon -> LDS
//                      positions, control / alignment / progress costs;
//   Gate-SDF decoder   over the tile's (rollout, step, gate) query rows in
//                      blocks of 16 rows, the hidden H x H layers on the matrix
//                      cores, every wave's weight slice resident in VGPRs for
//                      the whole kernel, activations passed through LDS;
//   tile partial       FP64 (rho_i, eta_i, eta2_i, S_i[T][4]) of the tile.
// A second kernel (one workgroup per solve) merges the partials in an order
// fixed by the tile index (results do not depend on which workgroup ran which
// tile or on what else was in the batch) and writes U*, the weights, the warm
// start and the tick.  The kernel boundary publishes the partials; a
// device-wide fence per tile instead costs tens of microseconds on a chip
// whose XCDs have separate L2 caches.
//
// Decoder schedule (8 waves).  With one hidden H x H layer every wave owns
// H/8 of its neurons; with two, waves 0-3 own H/4 neurons each of the first
// and waves 4-7 of the second.  Blocks of 16 rows flow through a software
// pipeline; in step s
//   wave 0          gate-frame points of block s+1
//   every wave      layer 1 of block s-1 or s, H/16 neuron blocks shared
//                   between the waves (FP32 matrix-core product with the
//                   point, then softplus)
//   owners of l     matrix-core products of layer l on block s-2-2l into one
//                   of two register accumulator sets, and the activation
//                   epilogue (softplus, bf16 split / output dot) of block
//                   s-3-2l from the other set
//   wave 3          output sum and max over gates of block s-2-2L
//                   (L hidden H x H layers)
// with one workgroup barrier per step.  A wave's products and its epilogue
// work on different blocks, so the matrix cores and the vector units overlap
// inside each wave.
//
// Precision variants of the hidden layers (FP32 accumulation throughout):
//   BF16    weights and activations rounded to bfloat16;
//   BF16X2  bfloat16 weights, activations split a = hi + lo (two products);
//   BF16X3  bfloat16 weights, a = hi + mid + lo exactly (three products);
//   F16X2   the bfloat16-rounded weights held exactly in FP16 under a
//           per-layer power-of-two scale, activations split a = hi + lo in
//           FP16 (two FP16 products, |a - hi - lo| <= 2^-22 |a| + 2^-25);
//   FP8     OCP E4M3 weights with a per-layer scale, E4M3 activations with a
//           static per-layer scale (saturating).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"
#include "ring.hpp"
#include "weights.hpp"

namespace mppi {

using f32x4 = __attribute__((ext_vector_type(4))) float;
using bf16x8 = __attribute__((ext_vector_type(8))) __bf16;
using bf16x2v = __attribute__((ext_vector_type(2))) __bf16;
using f16x8 = __attribute__((ext_vector_type(8))) _Float16;
using f16x2v = __attribute__((ext_vector_type(2))) _Float16;

constexpr int kWaves = 8;            // waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kTileR = 16;           // rollouts per tile
constexpr int kRows = 16;            // query rows per pipeline block
__host__ __device__ constexpr int kPartStride(int T) { return 4 + 4 * T; }

enum { P_BF16 = 1, P_BF16X2 = 2, P_FP8 = 3, P_BF16X3 = 4, P_F16X2 = 5 };

// splits: activation terms (one product each); fp8 / f16: operand type;
// scaled: the weights carry a per-layer scale.  FP8 starts the accumulators
// at zero and its epilogue forms scale * acc + bias; F16X2 (power-of-two
// scale 2^-s) starts them at 2^s bias, kept pre-scaled in LDS, and its
// epilogue forms scale * acc, both exact scalings; the bfloat16 kinds start
// them at the bias.
template <int P> struct PrecTraits;
template <int NS, bool F8, bool F16> struct PrecBase {
  static constexpr int splits = NS;
  static constexpr bool fp8 = F8, f16 = F16, scaled = F8 || F16;
};
template <> struct PrecTraits<P_BF16> : PrecBase<1, false, false> {};
template <> struct PrecTraits<P_BF16X2> : PrecBase<2, false, false> {};
template <> struct PrecTraits<P_BF16X3> : PrecBase<3, false, false> {};
template <> struct PrecTraits<P_FP8> : PrecBase<1, true, false> {};
template <> struct PrecTraits<P_F16X2> : PrecBase<2, false, true> {};

// max(x, 0) as one integer max on the bit pattern (negative floats, -0
// included, are negative integers); a float max would first quiet a
// possible signalling NaN, one more instruction per activation.
__device__ __forceinline__ float relu_bits(float x) {
  const int i = __float_as_int(x);
  return __int_as_float(i > 0 ? i : 0);
}

// softplus with the hardware base-2 exponential and logarithm:
// max(x, 0) + ln2 * log2(1 + 2^(-|x| log2 e)); absolute error ~1e-7.
__device__ __forceinline__ float softplus_fast(float x) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(x) * 1.4426950408889634f);
  return fmaf(__builtin_amdgcn_logf(1.0f + e), 0.6931471805599453f, relu_bits(x));
}

// softplus whose result stays within the finite half range: max(x, 0) is
// taken as min(max(x, 0), 65503) in one integer med3 on the bit pattern; the
// logarithmic term adds less than 2^-1000 there, so the result is at most
// 65503.  Differs from softplus only for x > 65503.
__device__ __forceinline__ float softplus_capped(float x) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(x) * 1.4426950408889634f);
  const int i = __float_as_int(x);
  const int r = i > 0 ? (i < 0x477FDF00 ? i : 0x477FDF00) : 0;   // 65503.0f
  return fmaf(__builtin_amdgcn_logf(1.0f + e), 0.6931471805599453f, __int_as_float(r));
}

// Activation that becomes the next layer's operand: F16X2 needs it within
// the half range.
template <int P>
__device__ __forceinline__ float softplus_act(float x) {
  if constexpr (PrecTraits<P>::f16) return softplus_capped(x);
  else return softplus_fast(x);
}

// Four softplus evaluations in the arithmetic of softplus_fast /
// softplus_capped (CAP), stage by stage: the four base-2 exponentials, then
// the four logarithms, then the four sums.  The stages are kept apart for
// the scheduler, so the four independent chains overlap their latencies
// instead of running one after another through one temporary.
template <bool CAP>
__device__ __forceinline__ void softplus4(const float (&x)[4], float (&v)[4]) {
  float e[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) e[i] = __builtin_amdgcn_exp2f(-fabsf(x[i]) * 1.4426950408889634f);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < 4; ++i) e[i] = __builtin_amdgcn_logf(1.0f + e[i]);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = __float_as_int(x[i]);
    const int r = CAP ? (b > 0 ? (b < 0x477FDF00 ? b : 0x477FDF00) : 0) : (b > 0 ? b : 0);
    v[i] = fmaf(e[i], 0.6931471805599453f, __int_as_float(r));
  }
}

// LDS activation row stride in elements (bf16) / bytes (fp8): the pad keeps
// 16-byte operand reads of 16 consecutive rows on distinct banks.
template <int H> __host__ __device__ constexpr int act_stride_bf16() { return H + 8; }
template <int H> __host__ __device__ constexpr int act_stride_fp8() { return H + 16; }

// Bytes of one activation buffer (all split terms) of kRows rows.
template <int P, int H>
__host__ __device__ constexpr size_t act_buf_bytes() {
  return PrecTraits<P>::fp8 ? (size_t)kRows * act_stride_fp8<H>()
                            : (size_t)PrecTraits<P>::splits * kRows * act_stride_bf16<H>() * 2;
}

// Feature table of one block for the encoded-point layer 1: two FP16 terms
// (hi, lo) of every feature, per term kRows rows of 32 k32 features plus a
// pad of 8 (16-byte operand reads of 16 rows on distinct banks).
__host__ __device__ constexpr int pe_row_halves(int k32) { return 32 * k32 + 8; }
__host__ __device__ constexpr size_t pe_slot_bytes(int k32) { return (size_t)2 * kRows * pe_row_halves(k32) * 2; }

struct FusedLds {
  size_t act, w1p, hb, wo, cf, rt, base, los, dp, field, pts, opart, jl, wt, fac, misc, xch, rot, feat, total;
};

// The activation buffers (input of hidden layer l, block parity p) share
// their space with the tile's control samples, which live only in the tile
// prologue (dynamics) and epilogue (weighted sums), outside the decoder.
template <int P, int H, int NHH>
__host__ __device__ FusedLds fused_lds(int Tm, int Gm, int max_tiles, int feat_ks = 0) {
  constexpr int WPL = kWaves / NHH;
  FusedLds L{};
  size_t o = 0;
  auto take = [&](size_t b) { const size_t r = o; o = (o + b + 15) / 16 * 16; return r; };
  const size_t acts = 2 * NHH * act_buf_bytes<P, H>();
  const size_t samp = sizeof(float) * 4 * kTileR * Tm;
  // fixed-size tables and the activation buffers first (compile-time
  // offsets for everything the decoder steps touch), then per-solve tables
  L.w1p = take(sizeof(float) * 4 * H);
  L.hb = take(sizeof(float) * NHH * H);
  L.wo = take(sizeof(float) * H);
  L.pts = take(sizeof(float) * 4 * kRows * 3);
  L.opart = take(sizeof(float) * 2 * WPL * kRows * 4);
  L.jl = take(sizeof(float) * 2 * kTileR);
  L.wt = take(sizeof(double) * (kTileR + 4));
  L.misc = take(64);
  L.rot = take(sizeof(float) * 8 * kTileR);
  L.act = take(acts > samp ? acts : samp);
  L.cf = take(sizeof(float) * Gm * H);
  L.rt = take(sizeof(float) * 9 * Gm);
  L.base = take(sizeof(float) * 3 * Gm * (Tm + 1));
  L.los = take(sizeof(float) * 2 * Tm);
  L.dp = take(sizeof(float) * 3 * kTileR * (Tm + 1));
  L.field = take(sizeof(float) * (kTileR * Tm + 1));   // + the reduction's sink entry
  L.fac = take(sizeof(double) * max_tiles);
  // positional encoding: three slots of the FP16 feature table
  L.feat = take(pe_slot_bytes(feat_ks) * 3);
  L.total = o;
  return L;
}

// Per-lane weight fragment of hidden layer l (A operand, 16x16x32): neuron
// block nb (16 neurons), K-step ks; the lane holds
// W[16 nb + lane % 16][32 ks + 8 (lane / 16) + j], j < 8.
// BF16: 16 bytes; FP8: 8 bytes.
template <int H>
__host__ __device__ constexpr size_t frag_index(int l, int nb, int ks, int lane) {
  return (((size_t)l * (H / 16) + nb) * (H / 32) + ks) * 64 + lane;
}

// Shared-memory views of one workgroup.
struct Views {
  char *act, *xch;
  float* rot;      // rotor-thrust-rate input: thrusts (4) and body rate (3) per rollout
  float *samp, *w1p, *hb, *wo, *cf, *rt, *base, *los, *dp, *field, *pts, *opart, *jl;
  char* feat;      // encoded-point features of three blocks (positional encoding only)
  double *wt, *fac;
  int* misc;
};

template <int P, int H, int NHH>
__device__ __forceinline__ Views make_views(char* lds, int Tm, int Gm, int max_tiles, int feat_ks = 0) {
  const FusedLds L = fused_lds<P, H, NHH>(Tm, Gm, max_tiles, feat_ks);
  Views v{};
  v.act = lds + L.act;
  v.samp = (float*)(lds + L.act);
  v.w1p = (float*)(lds + L.w1p);
  v.hb = (float*)(lds + L.hb);
  v.wo = (float*)(lds + L.wo);
  v.cf = (float*)(lds + L.cf);
  v.rt = (float*)(lds + L.rt);
  v.base = (float*)(lds + L.base);
  v.los = (float*)(lds + L.los);
  v.dp = (float*)(lds + L.dp);
  v.field = (float*)(lds + L.field);
  v.pts = (float*)(lds + L.pts);
  v.opart = (float*)(lds + L.opart);
  v.jl = (float*)(lds + L.jl);
  v.wt = (double*)(lds + L.wt);
  v.fac = (double*)(lds + L.fac);
  v.misc = (int*)(lds + L.misc);
  v.rot = (float*)(lds + L.rot);
  v.feat = lds + L.feat;
  return v;
}

// Two floats -> packed bfloat16 pair (round to nearest even), and back.
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const bf16x2v t = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, t);
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// The same for IEEE half precision (round to nearest even).
__device__ __forceinline__ uint32_t pack_f16(float a, float b) {
  const f16x2v t = {(_Float16)a, (_Float16)b};
  return __builtin_bit_cast(uint32_t, t);
}

// a - (half h of word w), in one mixed-precision FMA that reads the half
// straight from the packed word: exact, since the half is a's own rounding.
__device__ __forceinline__ float rem_f16_lo(uint32_t w, float a) {
  float r;
  asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(a));
  return r;
}
__device__ __forceinline__ float rem_f16_hi(uint32_t w, float a) {
  float r;
  asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(a));
  return r;
}

// Two-term half split of 4 activations in [0, 65503]: hi = RNE half of the
// value, lo = RNE half of the exact remainder; hi in h[0..1], lo in l[0..1]
// (two halves per word).  The values are kept opaque before the packing so
// that the compiler forms hi from the float32 activation (not from a fused
// re-evaluation of the softplus, one more instruction per pair).
__device__ __forceinline__ void split_f16(const float* v, uint32_t (&h)[2], uint32_t (&l)[2]) {
  float a[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    a[i] = v[i];
    asm("" : "+v"(a[i]));
  }
  h[0] = pack_f16(a[0], a[1]);
  h[1] = pack_f16(a[2], a[3]);
  l[0] = pack_f16(rem_f16_lo(h[0], a[0]), rem_f16_hi(h[0], a[1]));
  l[1] = pack_f16(rem_f16_lo(h[1], a[2]), rem_f16_hi(h[1], a[3]));
}

// Byte offset of (row n, neuron / K index m) inside one split term of an
// activation buffer, and the byte size of one split term.
template <int P, int H>
__host__ __device__ constexpr uint32_t act_off(int n, int m) {
  return PrecTraits<P>::fp8 ? (uint32_t)(n * act_stride_fp8<H>() + m) : (uint32_t)(n * act_stride_bf16<H>() + m) * 2u;
}
template <int P, int H>
__host__ __device__ constexpr uint32_t act_term_bytes() {
  return PrecTraits<P>::fp8 ? (uint32_t)(kRows * act_stride_fp8<H>()) : (uint32_t)(kRows * act_stride_bf16<H>() * 2);
}

// Write 4 consecutive neurons of one row, at byte offset `off` of activation
// buffer `buf`, as the operand of the next layer.  bf16 splits:
// a = hi + (mid) + (lo) with each term the round-to-nearest bfloat16 of the
// remainder; for three terms the sum is exact.
template <int P, int H>
__device__ __forceinline__ void put_act(char* buf, uint32_t off, const float v[4], float inv) {
  using PT = PrecTraits<P>;
  if constexpr (PT::fp8) {
    // saturate to the largest E4M3 value: the conversion alone turns values
    // beyond the last rounding interval into NaN (activations are >= 0)
    float q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = fminf(v[i] * inv, 448.0f);
    uint32_t word = __builtin_amdgcn_cvt_pk_fp8_f32(q[0], q[1], 0, false);
    word = __builtin_amdgcn_cvt_pk_fp8_f32(q[2], q[3], word, true);
    *(uint32_t*)(buf + off) = word;
  } else if constexpr (PT::f16) {
    uint32_t h[2], l[2];
    split_f16(v, h, l);
    *(uint2*)(buf + off) = make_uint2(h[0], h[1]);
    *(uint2*)(buf + off + act_term_bytes<P, H>()) = make_uint2(l[0], l[1]);
  } else {
    constexpr int NS = PT::splits;
    float r0 = v[0], r1 = v[1], r2 = v[2], r3 = v[3];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const uint32_t w01 = pack_bf16(r0, r1), w23 = pack_bf16(r2, r3);
      *(uint2*)(buf + off + s * act_term_bytes<P, H>()) = make_uint2(w01, w23);
      if (s + 1 < NS) {
        r0 -= bf16_lo(w01);
        r1 -= bf16_hi(w01);
        r2 -= bf16_lo(w23);
        r3 -= bf16_hi(w23);
      }
    }
  }
}

template <int P>
using FragT = typename std::conditional<PrecTraits<P>::fp8, long,
                                        typename std::conditional<PrecTraits<P>::f16, f16x8, bf16x8>::type>::type;

// One 16x16x32 matrix-core product of the precision's operand type.
template <int P>
__device__ __forceinline__ f32x4 mfma_lp(const FragT<P>& a, const FragT<P>& b, const f32x4& c) {
  if constexpr (PrecTraits<P>::fp8) return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
  else if constexpr (PrecTraits<P>::f16) return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Per-tile constants of the decoder's edge work (points and output
// reduction), read once per tile: the loop's scheduling fences would
// otherwise make every step reload them from the descriptor.  A block holds
// kRows / G positions of G gate rows each; this lane's row is position p,
// gate g of the block.
struct EdgeConsts {
  int G, T, Pc, qoff, npos, p, g;
  float invT, bout;
};

__device__ __forceinline__ EdgeConsts edge_consts(const SolveDesc& d, int lane, int npos, float bout) {
  EdgeConsts e;
  e.G = d.G;
  e.T = d.T;
  e.Pc = kRows / e.G;
  e.qoff = (int)d.q_off;
  e.npos = npos;
  e.p = lane / e.G;
  e.g = lane - e.p * e.G;
  e.invT = 1.0f / (float)e.T;
  e.bout = bout;
  return e;
}

// Gate-frame point of the row of block c that EdgeConsts e was made for, in
// two parts (the LDS reads, then the arithmetic and the store) so that a wave
// can issue the reads before other work and finish after it.  Branch-free:
// a padding row or a position past the tile reads position 0 and stores the
// zero point, so every lane of a wave may run it (lanes with the same row
// store the same value).
struct PointJob {
  float dp[3], r[9], b[3];
  bool ok;
  int gate;
  __device__ __forceinline__ void load(const Views& V, const EdgeConsts& e, int c) {
    const int q = c * e.Pc + e.p;
    ok = e.p < e.Pc && q < e.npos;
    gate = e.p < e.Pc ? e.g : 0;
    const int qv = ok ? q : 0;
    // q = kl T + t; (q + 1/2) / T is at least 1/(2T) away from an integer,
    // far more than the float error for q < 2^11
    const int kl = (int)(((float)qv + 0.5f) * e.invT), t = qv - kl * e.T;
    const int tp = t + e.qoff;
    const float* dpp = V.dp + 3 * (kl * (e.T + 1) + tp);
    const float* R = V.rt + 9 * e.g;
    const float* bb = V.base + 3 * (e.g * (e.T + 1) + tp);
#pragma unroll
    for (int i = 0; i < 3; ++i) { dp[i] = dpp[i]; b[i] = bb[i]; }
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = R[i];
  }
  __device__ __forceinline__ void store(float* out4) const {
    const float px = fmaf(r[0], dp[0], fmaf(r[1], dp[1], fmaf(r[2], dp[2], b[0])));
    const float py = fmaf(r[3], dp[0], fmaf(r[4], dp[1], fmaf(r[5], dp[2], b[1])));
    const float pz = fmaf(r[6], dp[0], fmaf(r[7], dp[1], fmaf(r[8], dp[2], b[2])));
    *(float4*)out4 = ok ? make_float4(px, py, pz, (float)gate) : make_float4(0.0f, 0.0f, 0.0f, (float)gate);
  }
};

__device__ __forceinline__ void chunk_point(const Views& V, const EdgeConsts& e, int c, float* out4) {
  PointJob j;
  j.load(V, e, c);
  j.store(out4);
}

// Coordinate comp of the gate-frame point of row r of block c, in the same
// arithmetic as chunk_point (0 for a padding row).
__device__ __forceinline__ float row_coord(const Views& V, const EdgeConsts& e, int c, int r, int comp) {
  const int p = r / e.G, g = r - p * e.G;
  const int q = c * e.Pc + p;
  if (p >= e.Pc || q >= e.npos) return 0.0f;
  const int kl = (int)(((float)q + 0.5f) * e.invT), t = q - kl * e.T;
  const int tp = t + e.qoff;
  const float* dpp = V.dp + 3 * (kl * (e.T + 1) + tp);
  const float* R = V.rt + 9 * g + 3 * comp;
  const float* b = V.base + 3 * (g * (e.T + 1) + tp);
  return fmaf(R[0], dpp[0], fmaf(R[1], dpp[1], fmaf(R[2], dpp[2], b[comp])));
}

// Encoded-point features (Section III-B) of block c's rows into one slot of
// the feature table: feature f = 3 + 6k + i is the sine (i < 3) or cosine
// (i >= 3) of pi 2^k times coordinate i mod 3, f < 3 the coordinates
// themselves; each is stored as hi = its RNE half and lo = the RNE half of
// the remainder, at [term][row][f] (row stride pe_row_halves).  Once per
// block for the whole workgroup: thread tid takes one raw coordinate
// (tid < 3 kRows) or one (row, coordinate, frequency) item with its sine and
// cosine; features past 3 + 6F stay at the zero they were cleared to.
__device__ __forceinline__ void put_feature(_Float16* t, int stride, int r, int f, float v) {
  const _Float16 hi = (_Float16)v;
  t[r * stride + f] = hi;
  t[kRows * stride + r * stride + f] = (_Float16)(v - (float)hi);
}
__device__ __forceinline__ void pe_block(const Views& V, const EdgeConsts& e, int c, char* slot, int F, int k32,
                                         int tid) {
  int r, comp, k = -1;
  if (tid < 3 * kRows) {
    r = tid / 3;
    comp = tid - 3 * r;
  } else {
    const int j = tid - 3 * kRows;
    if (j >= 3 * kRows * F) return;
    r = j / (3 * F);
    const int rem = j - r * 3 * F;
    k = rem / 3;
    comp = rem - 3 * k;
  }
  const float v = row_coord(V, e, c, r, comp);
  _Float16* t = (_Float16*)slot;
  const int stride = pe_row_halves(k32);
  if (k < 0) {
    put_feature(t, stride, r, comp, v);
  } else {
    float sn, cs;
    sincospif(ldexpf(v, k), &sn, &cs);
    put_feature(t, stride, r, 3 + 6 * k + comp, sn);
    put_feature(t, stride, r, 6 + 6 * k + comp, cs);
  }
}

// Value of lane perm(lane) under a DPP lane pattern (quad permutation or row
// mirror), every lane active.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Output of one row of block c: sum of the per-lane partials of the last
// layer's owners, max over each position's gates into the tile's field table
// (the hinge is taken in the tile epilogue).  Like PointJob in two parts and
// branch-free over the lanes (row = lane % 16, every 16-lane row of the wave
// a copy): a store that has no position (a block outside 0 .. nblk-1, a
// padding row, a gate other than the first) goes to the sink entry
// field[kTileR T], which no position uses.
template <int WPL>
struct ReduceJob {
  float4 o[WPL];
  __device__ __forceinline__ void load(const float* opart, int row) {
#pragma unroll
    for (int w = 0; w < WPL; ++w) o[w] = *(const float4*)(opart + 4 * (w * kRows + row));
  }
  __device__ __forceinline__ void store(const Views& V, const EdgeConsts& e, int c, int nblk) const {
    float acc = 0.0f;
#pragma unroll
    for (int w = 0; w < WPL; ++w) acc += (o[w].x + o[w].y) + (o[w].z + o[w].w);
    const float sv = acc + e.bout;
    float best = sv;
    if ((e.G & (e.G - 1)) == 0) {
      // G = 1, 2, 4, 8: a position's rows are an aligned group of G lanes;
      // maximum by lane exchanges inside the group (xor 1, xor 2 in a quad,
      // then the mirror of an 8-lane half row)
      if (e.G >= 2) best = fmaxf(best, dpp_f32<0xB1>(best));
      if (e.G >= 4) best = fmaxf(best, dpp_f32<0x4E>(best));
      if (e.G >= 8) best = fmaxf(best, dpp_f32<0x141>(best));
    } else {
      const int base = e.p * e.G + (__lane_id() & ~(kRows - 1));
      for (int g = 1; g < e.G; ++g) {
        const float x = __shfl(sv, base + g, 64);
        if (e.p * e.G + g < kRows) best = fmaxf(best, x);
      }
    }
    const int q = c * e.Pc + e.p;
    const bool ok = c >= 0 && c < nblk && e.g == 0 && e.p < e.Pc && q < e.npos;
    V.field[ok ? q : kTileR * e.T] = best;
  }
};

// Clipped control samples of the tile (Section IV-A) into V.samp.
__device__ __forceinline__ void tile_noise(const Views& V, const SolveDesc& d, int k0, int Re, uint32_t tick) {
  const int T = d.T;
  for (int i = threadIdx.x; i < Re * T; i += blockDim.x) {
    const int kl = i / T, t = i - kl * T;
    float u[4];
    sample_control(d, (uint32_t)(k0 + kl), (uint32_t)t, tick, u);
    *(float4*)(V.samp + 4 * i) = make_float4(u[0], u[1], u[2], u[3]);
  }
}

// Dynamics of this lane's rollout (lanes < Re): positions into V.dp and the
// rollout's progress + control + alignment cost into V.jl.  ROTOR: the
// rotor-thrust-rate input, whose extra state (thrusts, body rate) lives in
// LDS (V.rot) between steps: the decoder's weights occupy half the registers
// for the kernel's life, and rotor state in registers here would push other
// long-lived values into scratch memory for every tile.
template <bool ROTOR>
__device__ __forceinline__ void tile_dynamics(const Views& V, const SolveDesc& d, int tid) {
  const int T = d.T;
  RolloutState s;
#pragma unroll
  for (int i = 0; i < 3; ++i) { s.dp[i] = 0.0f; s.dv[i] = 0.0f; }
#pragma unroll
  for (int i = 0; i < 4; ++i) s.q[i] = d.q0[i];
  float* rsm = V.rot + 8 * tid;
  if constexpr (ROTOR) {
    RotorState rs;
    rotor_init(rs, d);
#pragma unroll
    for (int i = 0; i < 4; ++i) rsm[i] = rs.thr[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) rsm[4 + i] = rs.w[i];
  }
  float* dpk = V.dp + 3 * tid * (T + 1);
  dpk[0] = dpk[1] = dpk[2] = 0.0f;
  float Jc = 0.0f, Jv = 0.0f;
  const float4* su = (const float4*)(V.samp + 4 * tid * T);
  if constexpr (!ROTOR) {
    // The attitude increment of a step depends on its input only: the loop
    // forms the next step's increment beside this step's update, and reads
    // inputs two steps ahead, so that the serial chain per step is the state
    // update alone.
    float4 ua = su[0], ub = su[T > 1 ? 1 : 0];
    float r[4];
    {
      const float u0[4] = {ua.x, ua.y, ua.z, ua.w};
      quad_rotation(u0, d.dt, r);
    }
    for (int t = 0; t < T; ++t) {
      const float u[4] = {ua.x, ua.y, ua.z, ua.w};
      const float un[4] = {ub.x, ub.y, ub.z, ub.w};
      const float rc[4] = {r[0], r[1], r[2], r[3]};
      const RolloutState s0 = s;
      quad_advance(s, u[0], rc, d.dt, d.inv_mass, d.gravity);
      const float half = quad_rotation_series(un, d.dt, r);
      Jc = fmaf(u[0], u[0], fmaf(u[1], u[1], fmaf(u[2], u[2], fmaf(u[3], u[3], Jc))));
      dpk[3 * (t + 1) + 0] = s.dp[0];
      dpk[3 * (t + 1) + 1] = s.dp[1];
      dpk[3 * (t + 1) + 2] = s.dp[2];
      ua = ub;
      ub = su[t + 2 < T ? t + 2 : T - 1];
      quad_rotation_large(un, half, r);
      if (d.Q_vis != 0.0f) Jv += alignment_term(s0.q, V.los[2 * t] - s0.dp[0], V.los[2 * t + 1] - s0.dp[1]);
    }
  } else {
    // rotor input: the body rate, and with it the increment, is state
    for (int t = 0; t < T; ++t) {
      const float4 uu = su[t];
      const float u[4] = {uu.x, uu.y, uu.z, uu.w};
      Jc = fmaf(u[0], u[0], fmaf(u[1], u[1], fmaf(u[2], u[2], fmaf(u[3], u[3], Jc))));
      if (d.Q_vis != 0.0f) Jv += alignment_term(s.q, V.los[2 * t] - s.dp[0], V.los[2 * t + 1] - s.dp[1]);
      RotorState rs;
#pragma unroll
      for (int i = 0; i < 4; ++i) rs.thr[i] = rsm[i];
#pragma unroll
      for (int i = 0; i < 3; ++i) rs.w[i] = rsm[4 + i];
      float uc[4];
      rotor_step(rs, u, d, uc);
#pragma unroll
      for (int i = 0; i < 4; ++i) rsm[i] = rs.thr[i];
#pragma unroll
      for (int i = 0; i < 3; ++i) rsm[4 + i] = rs.w[i];
      quad_step(s, uc, d.dt, d.inv_mass, d.gravity);
      dpk[3 * (t + 1) + 0] = s.dp[0];
      dpk[3 * (t + 1) + 1] = s.dp[1];
      dpk[3 * (t + 1) + 2] = s.dp[2];
    }
  }
  const float Jg = s.dp[0] * s.dp[0] + s.dp[1] * s.dp[1] + s.dp[2] * s.dp[2] +
                   2.0f * (s.dp[0] * d.fprog[0] + s.dp[1] * d.fprog[1] + s.dp[2] * d.fprog[2]);
  V.jl[tid] = d.Q_gate * Jg + d.R_u * Jc + d.Q_vis * Jv;
}

// Dynamics of the tile's rollouts by scans over the horizon, for the
// collective-thrust + body-rate input, whose attitude increments depend on
// the input only (Section IV-A model; the same per-step arithmetic as
// quad_advance, summed in another order).  32 lanes per rollout (two
// rollouts per wave), lane l taking steps l C .. l C + C - 1, C = ceil(T/32):
//   attitude  q_t = q_0 (x) r_0 (x) ... (x) r_{t-1}: each lane multiplies its
//             chunk's increments, an exclusive scan over the lanes gives the
//             attitude at the chunk's start;
//   velocity  dv_t = sum_{s<t} a_s dt, a_s = (u_s,0 / m) R(q_s) e3 - g e3;
//   position  dp_t = sum_{s<t} (dv_s dt + a_s dt^2 / 2);
// each from an exclusive scan of the lanes' chunk sums, then the chunk's own
// steps in order.  Costs as in tile_dynamics.
struct Quat {
  float w, x, y, z;
};
__device__ __forceinline__ Quat qmul(const Quat& a, const Quat& b) {
  return Quat{a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
              a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
__device__ __forceinline__ float up32(float v, int dd) { return __shfl_up(v, (unsigned)dd, 32); }

// Exclusive prefix sum over the 32 lanes of each half-wave.
__device__ __forceinline__ float scan_excl32(float v, int l) {
#pragma unroll
  for (int dd = 1; dd < 32; dd <<= 1) {
    const float o = up32(v, dd);
    if (l >= dd) v += o;
  }
  const float e = up32(v, 1);
  return l == 0 ? 0.0f : e;
}

__device__ void tile_dynamics_scan(const Views& V, const SolveDesc& d, int Re) {
  const int tid = threadIdx.x, l = tid & 31, k = tid >> 5;
  const int T = d.T, C = (T + 31) >> 5;   // C <= 4 (T <= kMaxT = 128)
  const bool active = k < Re;
  const int kk = active ? k : 0;          // idle halves compute rollout 0 and store nothing
  const float4* su = (const float4*)(V.samp + 4 * kk * T);
  const int t0 = l * C;
  const float dt = d.dt, hdt2 = 0.5f * d.dt * d.dt, im = d.inv_mass, g = d.gravity;
  // increments of the chunk and their product; |u|^2 of its steps
  float r[4][4], f[4];
  float jc = 0.0f;
  Quat P{1.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int t = t0 + c;
    if (c < C && t < T) {
      const float4 uu = su[t];
      const float u[4] = {uu.x, uu.y, uu.z, uu.w};
      quad_rotation(u, dt, r[c]);
      f[c] = u[0] * im;
      jc = fmaf(u[0], u[0], fmaf(u[1], u[1], fmaf(u[2], u[2], fmaf(u[3], u[3], jc))));
    } else {
      r[c][0] = 1.0f;
      r[c][1] = r[c][2] = r[c][3] = 0.0f;
      f[c] = 0.0f;
    }
    P = qmul(P, Quat{r[c][0], r[c][1], r[c][2], r[c][3]});
  }
  // attitude at the chunk's start: q_0 (x) (exclusive product of the chunks before)
#pragma unroll
  for (int dd = 1; dd < 32; dd <<= 1) {
    const Quat o{up32(P.w, dd), up32(P.x, dd), up32(P.y, dd), up32(P.z, dd)};
    if (l >= dd) P = qmul(o, P);
  }
  Quat E{up32(P.w, 1), up32(P.x, 1), up32(P.y, 1), up32(P.z, 1)};
  if (l == 0) E = Quat{1.0f, 0.0f, 0.0f, 0.0f};
  const Quat qs = qmul(Quat{d.q0[0], d.q0[1], d.q0[2], d.q0[3]}, E);
  // accelerations of the chunk's steps and their sum
  float a[4][3], A[3] = {0.0f, 0.0f, 0.0f};
  {
    Quat q = qs;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float bx = 2.0f * (q.x * q.z + q.w * q.y);
      const float by = 2.0f * (q.y * q.z - q.w * q.x);
      const float bz = 1.0f - 2.0f * (q.x * q.x + q.y * q.y);
      const bool in = c < C && t0 + c < T;
      a[c][0] = in ? f[c] * bx : 0.0f;
      a[c][1] = in ? f[c] * by : 0.0f;
      a[c][2] = in ? fmaf(f[c], bz, -g) : 0.0f;
#pragma unroll
      for (int i = 0; i < 3; ++i) A[i] += a[c][i];
      q = qmul(q, Quat{r[c][0], r[c][1], r[c][2], r[c][3]});
    }
  }
  // velocity at the chunk's start, then the chunk's position increment
  float dv0[3], D[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int i = 0; i < 3; ++i) dv0[i] = scan_excl32(A[i], l) * dt;
  {
    float dv[3] = {dv0[0], dv0[1], dv0[2]};
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < C && t0 + c < T)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          D[i] += fmaf(a[c][i], hdt2, dv[i] * dt);
          dv[i] = fmaf(a[c][i], dt, dv[i]);
        }
  }
  float dp[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) dp[i] = scan_excl32(D[i], l);
  // the chunk's steps: positions out, alignment cost from the step-start state
  float* dpk = V.dp + 3 * k * (T + 1);
  if (active && l == 0) dpk[0] = dpk[1] = dpk[2] = 0.0f;
  float jv = 0.0f;
  {
    Quat q = qs;
    float dv[3] = {dv0[0], dv0[1], dv0[2]};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int t = t0 + c;
      if (c < C && t < T) {
        if (d.Q_vis != 0.0f) {
          const float qa[4] = {q.w, q.x, q.y, q.z};
          jv += alignment_term(qa, V.los[2 * t] - dp[0], V.los[2 * t + 1] - dp[1]);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          dp[i] = fmaf(a[c][i], hdt2, fmaf(dv[i], dt, dp[i]));
          dv[i] = fmaf(a[c][i], dt, dv[i]);
        }
        if (active) {
          dpk[3 * (t + 1) + 0] = dp[0];
          dpk[3 * (t + 1) + 1] = dp[1];
          dpk[3 * (t + 1) + 2] = dp[2];
        }
        q = qmul(q, Quat{r[c][0], r[c][1], r[c][2], r[c][3]});
      }
    }
  }
  // rollout sums over the 32 lanes (fixed butterfly) and the final position
#pragma unroll
  for (int m = 16; m >= 1; m >>= 1) {
    jc += __shfl_xor(jc, m, 32);
    jv += __shfl_xor(jv, m, 32);
  }
  const int ll = (T - 1) / C;              // lane holding the last step
  float pT[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) pT[i] = __shfl(dp[i], ll, 32);
  if (active && l == 0) {
    const float Jg = pT[0] * pT[0] + pT[1] * pT[1] + pT[2] * pT[2] +
                     2.0f * (pT[0] * d.fprog[0] + pT[1] * d.fprog[1] + pT[2] * d.fprog[2]);
    V.jl[k] = d.Q_gate * Jg + d.R_u * jc + d.Q_vis * jv;
  }
}

// Per-tile tables, noise and dynamics (all threads of the workgroup call it).
// The folded latent rows go to V.cf with row stride H + cf_pad.
__device__ void tile_prologue(const Views& V, const SolveDesc& d, int k0, int Re, uint32_t tick, int H,
                              int cf_pad = 0) {
  const int tid = threadIdx.x, T = d.T, G = d.G;
  for (int i = tid; i < G * H; i += (int)blockDim.x) V.cf[i + (cf_pad ? (i / H) * cf_pad : 0)] = d.cfold[i];
  for (int i = tid; i < 9 * G; i += (int)blockDim.x) V.rt[i] = d.Rt[i];
  for (int i = tid; i < 3 * G * (T + 1); i += (int)blockDim.x) V.base[i] = d.base[i];
  if (d.Q_vis != 0.0f)
    for (int i = tid; i < 2 * T; i += (int)blockDim.x) V.los[i] = d.los[i];
  tile_noise(V, d, k0, Re, tick);
  __syncthreads();
  // dynamics: rotor input one lane per rollout, serial over the horizon
  // (its body rate is state); collective thrust + body rate by scans
  if (d.dyn == 1) {
    if (tid < Re) tile_dynamics<true>(V, d, tid);
  } else {
    if (tid < 32 * kTileR) tile_dynamics_scan(V, d, Re);
  }
  __syncthreads();
}

// Sum over the 64 lanes of a wave by a fixed butterfly: every lane gets the
// same, schedule-independent result.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Per-rollout costs and the tile's FP64 partial (rho_i, eta_i, eta2_i,
// S_i[T][4]) with weights relative to the tile's own minimum.  The sums run in
// an order fixed by the rollout index.
__device__ void tile_epilogue(const Views& V, const SolveDesc& d, int k0, int Re, uint32_t tick) {
  const int tid = threadIdx.x, T = d.T;
  // the decoder reused the samples' space: draw them again (same counters)
  tile_noise(V, d, k0, Re, tick);
  {
    // hinge (eq. 7) summed over rollout k's T steps (eq. 8): blockDim / 16
    // (16 or 32) lanes per rollout, fixed butterfly; the field values go out
    // too when the solve asked for them
    const int lpr = blockDim.x / kTileR;
    const int k = tid / lpr, part = tid - k * lpr;
    float hs = 0.0f;
    for (int t = part; t < T; t += lpr) {
      const float sv = V.field[k * T + t];
      hs += fmaxf(0.0f, d.d_safe - sv);
      if (d.sdf && k < Re) d.sdf[(size_t)t * d.K + k0 + k] = sv;
    }
    for (int m = lpr / 2; m >= 1; m >>= 1) hs += __shfl_xor(hs, m, 64);
    if (part == 0 && k < Re) {
      const float J = V.jl[k] + d.Q_sdf * hs;
      V.jl[kTileR + k] = J;
      d.J[k0 + k] = J;
    }
  }
  __syncthreads();
  if (tid < kTileR) {
    double rho = INFINITY;
    for (int k = 0; k < Re; ++k) {
      const float J = V.jl[kTileR + k];
      if (isfinite(J)) rho = fmin(rho, (double)J);
    }
    const float J = tid < Re ? V.jl[kTileR + tid] : NAN;
    V.wt[tid] = (isfinite(J) && isfinite(rho)) ? exp(-((double)J - rho) * d.inv_lambda) : 0.0;
    if (tid == 0) V.wt[kTileR] = rho;
  }
  __syncthreads();
  if (tid == 0) {
    double eta = 0.0, eta2 = 0.0;
    for (int k = 0; k < kTileR; ++k) {
      eta += V.wt[k];
      eta2 += V.wt[k] * V.wt[k];
    }
    V.wt[kTileR + 1] = eta;
    V.wt[kTileR + 2] = eta2;
  }
  __syncthreads();
  double* part = d.partials + (size_t)(k0 / d.tile_rollouts) * kPartStride(T);
  if (tid < 3) part[tid] = V.wt[kTileR + tid];
  for (int i = tid; i < 4 * T; i += (int)blockDim.x) {
    double sacc = 0.0;
    for (int k = 0; k < Re; ++k) sacc = fma(V.wt[k], (double)V.samp[4 * (k * T) + i], sacc);
    part[4 + i] = sacc;
  }
}

// Ends a basic block: a branch on a value the compiler cannot see (always
// zero), with a memory clobber.  Code is not moved across it, so each part of
// a step keeps its place in the wave's instruction stream and its own
// register demand.
__device__ __forceinline__ void sched_fence() {
  int zz;
  asm volatile("s_mov_b32 %0, 0" : "=s"(zz) : : "memory");
  if (zz) asm volatile("s_nop 0");
}

template <int P>
using BFragT = FragT<P>;

// Pre-activation of one hidden neuron from its accumulator (see PrecBase).
template <int P>
__device__ __forceinline__ float pre_act(float acc, float scale, float bias) {
  if constexpr (PrecTraits<P>::fp8) return fmaf(acc, scale, bias);
  else if constexpr (PrecTraits<P>::f16) return acc * scale;
  else return acc;
}

// Hidden-layer bias as the accumulators' start value (F16X2: times 2^s).
template <int P>
__device__ __forceinline__ float bias_start(float b, float scale) {
  if constexpr (PrecTraits<P>::f16) return b / scale;
  else return b;
}

// B operands (16 rows x 32 K of every split term) of K-step ks from `in`;
// `off` is the lane's byte offset act_off(row, 8 (lane / 16)).
template <int P, int H>
__device__ __forceinline__ void read_operands(const char* in, uint32_t off, int ks,
                                              BFragT<P> (&b)[PrecTraits<P>::splits]) {
  constexpr int NS = PrecTraits<P>::splits;
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) {
    if constexpr (PrecTraits<P>::fp8) b[sp] = *(const long*)(in + off + 32 * ks);
    else b[sp] = __builtin_bit_cast(BFragT<P>, *(const uint4*)(in + off + sp * act_term_bytes<P, H>() + 64 * ks));
  }
}

// Matrix-core part of a step: acc = bias + W(owned) x in^T for 16 rows, one
// scheduling region per K-step with the next K-step's operands read ahead.
// b0 holds the operands of K-step 0 on entry.
template <int P, int H, int OWN, int MB>
__device__ __forceinline__ void products(const char* in, uint32_t boff, const float* hb, int gw, int h,
                                         const FragT<P> (&wreg)[MB][H / 32], BFragT<P> (&b0)[PrecTraits<P>::splits],
                                         f32x4 (&acc)[MB]) {
  using PT = PrecTraits<P>;
  constexpr int NS = PT::splits;
  constexpr int KS = H / 32;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    if constexpr (PT::fp8) acc[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    else acc[mb] = *(const f32x4*)(hb + OWN * H + 16 * (gw * MB + mb) + 4 * h);
  }
  BFragT<P> bn[NS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    if (ks + 1 < KS) read_operands<P, H>(in, boff, ks + 1, bn);
#pragma unroll
    for (int sp = 0; sp < NS; ++sp)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        acc[mb] = mfma_lp<P>(wreg[mb][ks], b0[sp], acc[mb]);
      }
#pragma unroll
    for (int sp = 0; sp < NS; ++sp) b0[sp] = bn[sp];
    sched_fence();
  }
}

// Layer 1: FP32 16x16x4 matrix-core products (A = W1[:, 0..2] of 16 neurons
// with a zero fourth column, B = the 16 rows' gate-frame points (x, y, z,
// gate), C = the folded latent term of each row's gate), then softplus.  The
// H/16 neuron blocks are split between the waves so that the two phases of a
// SIMD's pair of waves take about equally long: a products-first wave takes
// kL1B blocks (its products join the end of its matrix-core phase), a
// vector-first wave kL1A blocks (products at the start of its vector phase).
// With split activations (BF16X2/BF16X3/F16X2) the vector-first waves of a
// two-hidden-layer decoder carry the costly operand splits of the first
// hidden layer, so the products-first waves take 3 of every 4 layer-1
// blocks; with one activation term (BF16, FP8) the split is one conversion
// and the blocks are shared equally.  The two vector-first waves that carry
// the edge work (waves 0 and 3) hand one block each to the other two.
template <int P, int H> struct L1Split {
  static constexpr int B = (H >= 256 && PrecTraits<P>::splits > 1) ? 3 : H / 16 / kWaves;  // per products-first wave
  static constexpr int A = (H / 16 - (kWaves / 2) * B) / (kWaves / 2);
  static_assert(A >= 0 && (kWaves / 2) * (A + B) * 16 == H, "layer-1 split");
  static constexpr int S = A >= 1 ? 1 : 0;
  // blocks of a vector-first wave with (EDGE) or without edge work
  static constexpr int vf(bool edge) { return edge ? A - S : A + S; }
  // first block of wave w (waves 4-7 products first, 0-3 vector first; the
  // vector-first counts are A - S, A + S, A + S, A - S)
  __device__ static int first(int wave) {
    return wave >= kWaves / 2 ? (wave - kWaves / 2) * B
                              : (kWaves / 2) * B + wave * A + (wave == 1 ? -S : wave == 3 ? S : 0);
  }
  static_assert(kWaves == 8, "vector-first waves 0-3 with edge work on waves 0 and 3");
};

// PE (positional encoding, Section III-B): the point enters as PE(p), a
// product over K = 32 feat_k32 features on FP16 matrix cores with both
// operands split in two terms, W1' = W1 / scale = Wh + Wl and f = fh + fl:
// Wh fh + Wh fl + Wl fh (the dropped Wl fl and the term roundings leave
// ~2^-21 of |W1| |f| per feature).  The B operands come from the block's
// slot fs of the feature table, the A operands are fragments in global
// memory read through the caches (26 KB at H = 256); the accumulators start
// at the folded latent term / scale and end times scale (exact powers of 2).
template <int H, int NB, bool PE>
__device__ __forceinline__ void layer1_products(const float* pts, const char* fs, const float* cf, const float* w1p,
                                                int b0, int h, int nl, f32x4 (&x)[NB > 0 ? NB : 1],
                                                const DeviceWeights& w) {
  const int g = (int)pts[4 * nl + 3];
  if constexpr (!PE) {
    const float bk = pts[4 * nl + h];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const float4 c4 = *(const float4*)(cf + g * H + 16 * (b0 + j) + 4 * h);
      x[j] = f32x4{c4.x, c4.y, c4.z, c4.w};
      x[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(w1p[4 * (16 * (b0 + j) + nl) + h], bk, x[j], 0, 0, 0);
    }
  } else {
    const float sc = w.w1pe_scale, up = 1.0f / sc;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const float4 c4 = *(const float4*)(cf + g * H + 16 * (b0 + j) + 4 * h);
      x[j] = f32x4{c4.x * up, c4.y * up, c4.z * up, c4.w * up};
    }
    const int K32 = w.feat_k32, lane = 16 * h + nl, stride = pe_row_halves(K32);
    const uint4* wf = (const uint4*)w.w1pe16;
    for (int ks = 0; ks < K32; ++ks) {
      const char* rb = fs + (size_t)(nl * stride + 32 * ks + 8 * h) * 2;
      const f16x8 fh = __builtin_bit_cast(f16x8, *(const uint4*)rb);
      const f16x8 fl = __builtin_bit_cast(f16x8, *(const uint4*)(rb + (size_t)kRows * stride * 2));
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const size_t fi = (((size_t)(b0 + j) * K32 + ks) * 2) * 64 + lane;
        const f16x8 wh = __builtin_bit_cast(f16x8, wf[fi]);
        const f16x8 wl = __builtin_bit_cast(f16x8, wf[fi + 64]);
        x[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wh, fh, x[j], 0, 0, 0);
        x[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wh, fl, x[j], 0, 0, 0);
        x[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wl, fh, x[j], 0, 0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) x[j] = x[j] * sc;
  }
}

// Edge work that a vector-first wave carries inside its vector phase: the
// LDS reads are issued before the softplus of the owned layer and the result
// stored after it, so that the read latency hides behind the vector work.
struct NoEdge {
  __device__ __forceinline__ void load() {}
  __device__ __forceinline__ void store() const {}
};
struct PointEdge {      // gate-frame points of block c into slot `out`
  const Views& V;
  const EdgeConsts& e;
  int c;
  float* out;
  PointJob j;
  __device__ __forceinline__ void load() { j.load(V, e, c); }
  __device__ __forceinline__ void store() const { j.store(out + 4 * (__lane_id() & (kRows - 1))); }
};
template <int WPL>
struct ReduceEdge {     // output reduction of block c from the partials `opart`
  const Views& V;
  const EdgeConsts& e;
  const float* opart;
  int c, nblk;
  ReduceJob<WPL> j;
  __device__ __forceinline__ void load() { j.load(opart, __lane_id() & (kRows - 1)); }
  __device__ __forceinline__ void store() const { j.store(V, e, c, nblk); }
};

// Vector part of a step: the epilogue of the owned layer from acc (softplus,
// then the next layer's operand in `out`, or for the last layer this lane's
// share of the output dot in `opart`), and softplus and operand of the
// wave's NB layer-1 blocks x (first block b0) into `l1out`.
template <int P, int H, int NHH, int OWN, int MB, int NB, class EG>
__device__ __forceinline__ void vector_work(const f32x4 (&acc)[MB], const f32x4 (&x)[NB > 0 ? NB : 1], char* out,
                                            char* l1out, float* opart, const float* hb, const float* wo,
                                            const DeviceWeights& w, int b0, int gw, int h, int nl, float scale_own,
                                            EG& edge) {
  using PT = PrecTraits<P>;
  const int e0 = 16 * gw * MB + 4 * h;          // first owned neuron of this lane
  const uint32_t eoff = act_off<P, H>(nl, e0);
  float op = 0.0f;
  edge.load();
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    float xs[4], v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      xs[i] = pre_act<P>(acc[mb][i], scale_own, PT::fp8 ? hb[OWN * H + e0 + 16 * mb + i] : 0.0f);
    softplus4<OWN + 1 < NHH && PT::f16>(xs, v);
    if constexpr (OWN + 1 < NHH) {
      put_act<P, H>(out, eoff + act_off<P, H>(0, 16 * mb), v, PT::fp8 ? w.a_inv[OWN + 1] : 1.0f);
    } else {
      const float4 o4 = *(const float4*)(wo + e0 + 16 * mb);
      op = fmaf(o4.x, v[0], fmaf(o4.y, v[1], fmaf(o4.z, v[2], fmaf(o4.w, v[3], op))));
    }
    if (mb & 1) sched_fence();
  }
  edge.store();
  if constexpr (OWN + 1 == NHH) opart[(gw * kRows + nl) * 4 + h] = op;
  const uint32_t loff = act_off<P, H>(nl, 16 * b0 + 4 * h);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const float xs[4] = {x[j][0], x[j][1], x[j][2], x[j][3]};
    float v[4];
    softplus4<PT::f16>(xs, v);
    put_act<P, H>(l1out, loff + act_off<P, H>(0, 16 * j), v, PT::fp8 ? w.a_inv[0] : 1.0f);
    if (j & 1) sched_fence();
  }
}

// One pipeline step (see the schedule at the top) of a wave that owns hidden
// layer OWN; PAR is the parity of the step index.  The products of block
// s-2-2 OWN read activation buffer (OWN, PAR) into acc[PAR]; the epilogue of
// block s-3-2 OWN reads acc[1-PAR] (the previous step's products) and writes
// buffer (OWN+1, 1-PAR) or the output partials of parity 1-PAR; layer 1 of
// block s-1 goes to buffer (0, 1-PAR).  The two waves that share a SIMD run
// the two parts in opposite order (MFIRST: products first), so that one
// wave's matrix-core work runs beside the other's vector work.  Blocks outside
// the tile's range run on stale data whose results are never read.
template <int P, int H, int NHH, int OWN, int PAR, bool MFIRST, int MB, bool PE, int NBV, class EG>
__device__ __forceinline__ void pipeline_step(const Views& V, const DeviceWeights& w, int wave, int gw, int h,
                                              int nl, float scale_own, const FragT<P> (&wreg)[MB][H / 32],
                                              f32x4 (&acc)[2][MB], const float* pts_prev, const float* pts_cur,
                                              const char* fs_prev, const char* fs_cur,
                                              f32x4 (&x1c)[NBV > 0 ? NBV : 1], EG& edge) {
  constexpr int WPL = kWaves / NHH;
  constexpr size_t AB = act_buf_bytes<P, H>();
  const char* in = V.act + (2 * OWN + PAR) * AB;
  char* out = V.act + (2 * (OWN + 1 < NHH ? OWN + 1 : 0) + 1 - PAR) * AB;
  char* l1out = V.act + (1 - PAR) * AB;
  float* op = V.opart + (1 - PAR) * WPL * kRows * 4;
  const uint32_t boff = act_off<P, H>(nl, 8 * h);
  BFragT<P> b0[PrecTraits<P>::splits];
  const int l1b = L1Split<P, H>::first(wave);
  if constexpr (MFIRST) {
    // matrix-core phase: owned layer, then this wave's layer-1 blocks of
    // block s-1; vector phase after it
    constexpr int NB = L1Split<P, H>::B;
    f32x4 x1[NB > 0 ? NB : 1];
    read_operands<P, H>(in, boff, 0, b0);
    products<P, H, OWN, MB>(in, boff, V.hb, gw, h, wreg, b0, acc[PAR]);
    layer1_products<H, NB, PE>(pts_prev, fs_prev, V.cf, V.w1p, l1b, h, nl, x1, w);
    sched_fence();
    vector_work<P, H, NHH, OWN, MB, NB>(acc[1 - PAR], x1, out, l1out, op, V.hb, V.wo, w, l1b, gw, h, nl, scale_own, edge);
  } else {
    // vector phase (layer-1 products of block s-1 carried from the previous
    // step), then the matrix-core phase, which ends with the layer-1
    // products of block s for the next step: no matrix-core instruction in
    // the vector phase, where it would queue behind the other wave's products
    constexpr int NB = NBV;
    read_operands<P, H>(in, boff, 0, b0);
    vector_work<P, H, NHH, OWN, MB, NB>(acc[1 - PAR], x1c, out, l1out, op, V.hb, V.wo, w, l1b, gw, h, nl, scale_own,
                                        edge);
    sched_fence();
    products<P, H, OWN, MB>(in, boff, V.hb, gw, h, wreg, b0, acc[PAR]);
    layer1_products<H, NB, PE>(pts_cur, fs_cur, V.cf, V.w1p, l1b, h, nl, x1c, w);
  }
}

// The decoder over one tile's blocks for a wave that owns hidden layer OWN.
// Activation buffer (l, p) is the input of hidden layer l for blocks of
// parity p.  Every wave runs the same number of steps and barriers.
template <int P, int H, int NHH, int OWN, bool MFIRST, int MB, bool PE, int EDGE>
__device__ __forceinline__ void decoder_tile(const Views& V, const SolveDesc& d, const DeviceWeights& w, int wave,
                                             int lane, int gw, int h, int nl, float scale_own,
                                             const FragT<P> (&wreg)[MB][H / 32], int npos, int nblk) {
  constexpr int WPL = kWaves / NHH;
  constexpr int lag = 2 + 2 * NHH;    // step at which a block's output is reduced
  const int nsteps = nblk + lag;
  f32x4 acc[2][MB];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[p][mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  constexpr int NBV = L1Split<P, H>::vf(EDGE != 0);   // layer-1 blocks of a vector-first wave
  f32x4 x1c[NBV > 0 ? NBV : 1];
#pragma unroll
  for (int j = 0; j < (NBV > 0 ? NBV : 1); ++j) x1c[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  // Gate-frame points of block b live in slot b % 3: in step s one wave
  // (EDGE 1) writes block s+1 while the layer-1 products read blocks s-1 and
  // s, and another (EDGE 2) reduces the output of block s - lag.  Both are
  // vector-first waves on different SIMDs, which finish their own work
  // earliest; they run the edge work inside their vector phase.
  // With the positional encoding every thread also forms its share of the
  // features of block s+1 in step s, into feature slot (s+1) % 3.
  const EdgeConsts ec = edge_consts(d, lane & (kRows - 1), npos, w.bout);
  const size_t fslot = pe_slot_bytes(w.feat_k32);
  if (EDGE == 1 && lane < kRows) chunk_point(V, ec, 0, V.pts + 4 * lane);
  if constexpr (PE) pe_block(V, ec, 0, V.feat, w.pe_freqs, w.feat_k32, 64 * wave + lane);
  __syncthreads();
  int slot = 0;                       // = s % 3
  auto edges = [&](int st) {
    if constexpr (PE) {
      const int nxt = slot == 2 ? 0 : slot + 1;
      pe_block(V, ec, st + 1, V.feat + nxt * fslot, w.pe_freqs, w.feat_k32, 64 * wave + lane);
    }
  };
  auto edge_job = [&](int st, int par) {
    if constexpr (EDGE == 1) {
      const int nxt = slot == 2 ? 0 : slot + 1;
      return PointEdge{V, ec, st + 1, V.pts + 4 * kRows * nxt, {}};
    } else if constexpr (EDGE == 2) {
      return ReduceEdge<WPL>{V, ec, V.opart + par * WPL * kRows * 4, st - lag, nblk, {}};
    } else {
      return NoEdge{};
    }
  };
  auto slot_pts = [&](int sl) { return V.pts + 4 * kRows * sl; };
  auto slot_fs = [&](int sl) { return V.feat + fslot * sl; };
  for (int s = 0; s < nsteps; s += 2) {
    // the lane indices pass through an empty asm each step, so the compiler
    // recomputes the lane's LDS addresses inside the step (a few adds)
    // instead of keeping a dozen of them live across the loop
    int hv = h, nv = nl;
    asm volatile("" : "+v"(hv), "+v"(nv));
    edges(s);
    {
      auto ej = edge_job(s, 0);
      pipeline_step<P, H, NHH, OWN, 0, MFIRST, MB, PE, NBV>(V, w, wave, gw, hv, nv, scale_own, wreg, acc,
                                                   slot_pts(slot == 0 ? 2 : slot - 1), slot_pts(slot),
                                                   slot_fs(slot == 0 ? 2 : slot - 1), slot_fs(slot), x1c, ej);
    }
    __syncthreads();
    slot = slot == 2 ? 0 : slot + 1;
    asm volatile("" : "+v"(hv), "+v"(nv));
    edges(s + 1);
    {
      auto ej = edge_job(s + 1, 1);
      pipeline_step<P, H, NHH, OWN, 1, MFIRST, MB, PE, NBV>(V, w, wave, gw, hv, nv, scale_own, wreg, acc,
                                                   slot_pts(slot == 0 ? 2 : slot - 1), slot_pts(slot),
                                                   slot_fs(slot == 0 ? 2 : slot - 1), slot_fs(slot), x1c, ej);
    }
    __syncthreads();
    slot = slot == 2 ? 0 : slot + 1;
  }
}

// The steps of k_fused below as functions, for the served ring kernel
// (k_fused keeps them written out).  Once per kernel: the weights of the
// owned neurons into VGPRs (resident for the whole kernel) and the small
// per-network tables into LDS; returns the owned layer's scale.
template <int P, int H, int NHH, bool PE, int MB>
__device__ __forceinline__ float fused_setup(const Views& V, const DeviceWeights& w, int tid, int lane, int own,
                                             int gw, FragT<P> (&wreg)[MB][H / 32]) {
  using PT = PrecTraits<P>;
  // feature table: padding features (past 3 + 6F) must read as zero
  if constexpr (PE)
    for (int i = tid; i < (int)(3 * pe_slot_bytes(w.feat_k32) / 4); i += kThreads) ((uint32_t*)V.feat)[i] = 0u;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int ks = 0; ks < H / 32; ++ks) {
      const size_t fi = frag_index<H>(own, gw * MB + mb, ks, lane);
      if constexpr (PT::fp8) wreg[mb][ks] = ((const long*)w.hidden_lp)[fi];
      else wreg[mb][ks] = __builtin_bit_cast(FragT<P>, ((const uint4*)w.hidden_lp)[fi]);
    }
  const float scale_own = PT::scaled ? w.w_scale[own] * w.a_scale[own] : 1.0f;
  for (int i = tid; i < 4 * H; i += kThreads) V.w1p[i] = w.w1p[i];
  for (int i = tid; i < NHH * H; i += kThreads) V.hb[i] = bias_start<P>(w.hbias[i], PT::scaled ? w.w_scale[i / H] : 1.0f);
  for (int i = tid; i < H; i += kThreads) V.wo[i] = w.wout[i];
  return scale_own;
}

// One tile: the 16 rollouts of solve d from rollout k0 (noise, dynamics,
// decoder, costs, the tile's FP64 partial); every thread of the workgroup.
template <int P, int H, int NHH, bool PE, int MB>
__device__ __forceinline__ void fused_tile(const Views& V, const SolveDesc& d, const DeviceWeights& w, int k0,
                                           int wave, int lane, int gw, int h, int nl, float scale_own,
                                           const FragT<P> (&wreg)[MB][H / 32]) {
  const int K = d.K, T = d.T, G = d.G;
  const int Re = min(kTileR, K - k0);
  const uint32_t tick = d.tick_fixed == 0xFFFFFFFFu ? *d.tick_slot : d.tick_fixed;
  tile_prologue(V, d, k0, Re, tick, H);
  const int npos = Re * T;
  const int nblk = (npos + kRows / G - 1) / (kRows / G);
  // waves w and w + 4 share a SIMD: the second runs its products first
  // (with two hidden layers that is the owner of the last one, whose
  // epilogue needs the fewest registers beside two accumulator sets)
  // (waves 0 and kWaves / 2 - 1, vector first, also carry the edge work)
  if (wave >= kWaves / 2)
    decoder_tile<P, H, NHH, NHH - 1, true, MB, PE, 0>(V, d, w, wave, lane, gw, h, nl, scale_own, wreg, npos, nblk);
  else if (wave == 0)
    decoder_tile<P, H, NHH, 0, false, MB, PE, 1>(V, d, w, wave, lane, gw, h, nl, scale_own, wreg, npos, nblk);
  else if (wave == kWaves / 2 - 1)
    decoder_tile<P, H, NHH, 0, false, MB, PE, 2>(V, d, w, wave, lane, gw, h, nl, scale_own, wreg, npos, nblk);
  else
    decoder_tile<P, H, NHH, 0, false, MB, PE, 0>(V, d, w, wave, lane, gw, h, nl, scale_own, wreg, npos, nblk);
  tile_epilogue(V, d, k0, Re, tick);
}

template <int P, int H, int NHH, bool PE>
__global__ __launch_bounds__(kThreads, 1) void k_fused(FusedBatch batch, DeviceWeights w, int Tm, int Gm,
                                                        int max_tiles) {
  using PT = PrecTraits<P>;
  constexpr int WPL = kWaves / NHH;   // waves per hidden layer
  constexpr int MB = H / WPL / 16;    // 16-neuron blocks per wave
  constexpr int KS = H / 32;          // K-steps of 32
  extern __shared__ __align__(16) char lds[];
  const Views V = make_views<P, H, NHH>(lds, Tm, Gm, max_tiles, PE ? w.feat_k32 : 0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 4, nl = lane & 15;
  const int own = wave / WPL, gw = wave % WPL;
  // feature table: padding features (past 3 + 6F) must read as zero
  if constexpr (PE)
    for (int i = tid; i < (int)(3 * pe_slot_bytes(w.feat_k32) / 4); i += kThreads) ((uint32_t*)V.feat)[i] = 0u;

  // ---- weights of the owned neurons, resident in VGPRs for the whole kernel
  FragT<P> wreg[MB][KS];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const size_t fi = frag_index<H>(own, gw * MB + mb, ks, lane);
      if constexpr (PT::fp8) wreg[mb][ks] = ((const long*)w.hidden_lp)[fi];
      else wreg[mb][ks] = __builtin_bit_cast(FragT<P>, ((const uint4*)w.hidden_lp)[fi]);
    }
  const float scale_own = PT::scaled ? w.w_scale[own] * w.a_scale[own] : 1.0f;
  for (int i = tid; i < 4 * H; i += kThreads) V.w1p[i] = w.w1p[i];
  for (int i = tid; i < NHH * H; i += kThreads) V.hb[i] = bias_start<P>(w.hbias[i], PT::scaled ? w.w_scale[i / H] : 1.0f);
  for (int i = tid; i < H; i += kThreads) V.wo[i] = w.wout[i];

  while (true) {
    __syncthreads();
    if (tid == 0) V.misc[0] = (int)atomicAdd(batch.tile_counter, 1u);
    __syncthreads();
    // uniform across the workgroup: descriptor reads go to scalar registers
    const int tile = __builtin_amdgcn_readfirstlane(V.misc[0]);
    if (tile >= batch.n_tiles) break;
    const int2 tl0 = batch.tiles[tile];
    const int2 tl = make_int2(__builtin_amdgcn_readfirstlane(tl0.x), __builtin_amdgcn_readfirstlane(tl0.y));
    const SolveDesc& d = batch.descs[tl.x];
    const int K = d.K, T = d.T, G = d.G;
    const int k0 = tl.y;
    const int Re = min(kTileR, K - k0);
    const uint32_t tick = d.tick_fixed == 0xFFFFFFFFu ? *d.tick_slot : d.tick_fixed;
    tile_prologue(V, d, k0, Re, tick, H);
    const int npos = Re * T;
    const int nblk = (npos + kRows / G - 1) / (kRows / G);
    // waves w and w + 4 share a SIMD: the second runs its products first
    // (with two hidden layers that is the owner of the last one, whose
    // epilogue needs the fewest registers beside two accumulator sets)
    // (waves 0 and kWaves / 2 - 1, vector first, also carry the edge work)
    if (wave >= kWaves / 2)
      decoder_tile<P, H, NHH, NHH - 1, true, MB, PE, 0>(V, d, w, wave, lane, gw, h, nl, scale_own, wreg, npos, nblk);
    else if (wave == 0)
      decoder_tile<P, H, NHH, 0, false, MB, PE, 1>(V, d, w, wave, lane, gw, h, nl, scale_own, wreg, npos, nblk);
    else if (wave == kWaves / 2 - 1)
      decoder_tile<P, H, NHH, 0, false, MB, PE, 2>(V, d, w, wave, lane, gw, h, nl, scale_own, wreg, npos, nblk);
    else
      decoder_tile<P, H, NHH, 0, false, MB, PE, 0>(V, d, w, wave, lane, gw, h, nl, scale_own, wreg, npos, nblk);
    tile_epilogue(V, d, k0, Re, tick);
  }
}

// Before the fused kernel: zero the batch's work counter and fold the
// latent block of every gate of every solve (workgroup (g, solve)).
__global__ __launch_bounds__(256) void k_fused_prep(FusedBatch b, DeviceWeights w) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *b.tile_counter = 0u;
  fold_gate(b.descs[blockIdx.y], blockIdx.x, w);
}

constexpr int kMergeThreads = 1024;
constexpr int kMergeSlice = 32;      // U* entries per merge workgroup (at most)

// Merge workgroups of a solve: each takes a slice of the 4T entries of U*
// (and of the K normalised weights).  A function of the solve alone, so the
// summation order below never depends on the rest of the batch.
__host__ __device__ constexpr int merge_groups(int T) { return (4 * T + kMergeSlice - 1) / kMergeSlice; }

// Merge of one solve's tile partials (runs after the fused kernel, whose
// completion makes every partial visible); workgroup (solve, c):
//   rho = min_i rho_i, f_i = exp(-(rho_i - rho) / lambda),
//   eta = sum_i eta_i f_i, U*[t][c] = sum_i S_i[t][c] f_i / eta,
// every workgroup forming rho, f and eta itself (the same values, in the same
// order), then its slice of U* and of the normalised weights; workgroup 0
// also the warm-start end, the tick and the scalars.  The U* sums run over
// C consecutive tile ranges, each summed in tile order, then the ranges in
// order, with C a function of T and the tile count only: the result does not
// depend on which workgroup ran which tile or on what else was in the batch.
// Merge group c of solve d on a workgroup of NT threads (NT = kMergeThreads,
// or fewer: then each thread plays kMergeThreads / NT of the threads above,
// and every sum keeps the order of kMergeThreads threads, so the result is
// the same bit for bit).  `lds` holds 3 kMergeThreads / 64 + kMergeThreads
// doubles, `fac` the solve's n tile factors.
template <int NT>
__device__ void merge_group(const SolveDesc& d, int c, double* lds, double* fac, bool reuse = false) {
  constexpr int VT = kMergeThreads;   // threads whose summation order is kept
  constexpr int NW = VT / 64;
  constexpr int R = VT / NT;
  static_assert(VT % NT == 0 && NT % 64 == 0, "whole waves");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = d.n_tiles, T = d.T, K = d.K;
  const int ng = merge_groups(T);
  const int nU = 4 * T, L = (nU + ng - 1) / ng, u0 = c * L, u1 = min(nU, u0 + L);
  const int C = max(1, min(n, VT / L));    // tile ranges of the U* sums
  double* red = lds;                  // 3 NW per-wave partial results
  double* part = red + 3 * NW;        // C x L partial sums of the slice
  // Reads that do not depend on rho go out first, so that their latency
  // passes during the reductions: this thread's U* item (tile range rg,
  // entry o; C L <= VT, so at most one) up to kPre of its tiles, and the
  // first of its costs for the weights (one thread per virtual thread only).
  constexpr int kPre = R == 1 ? 16 : 1;
  const int rg = tid / L, o = u0 + (tid - rg * L);
  const int j0 = rg * n / C, j1 = tid < C * L ? (rg + 1) * n / C : j0;
  const bool item = tid < C * L && o < u1;
  double sv[kPre];
#pragma unroll
  for (int q = 0; q < kPre; ++q) sv[q] = (R == 1 && item && j0 + q < j1) ? d.partials[(size_t)(j0 + q) * kPartStride(T) + 4 + o] : 0.0;
  const int kb = (int)((long)K * c / ng), ke = (int)((long)K * (c + 1) / ng);
  const float J0 = (R == 1 && (d.wn || d.J_copy) && kb + tid < ke) ? d.J[kb + tid] : 0.0f;
  // rho = min over tiles with weight (min is exact in any order); with
  // reuse, rho, the tile factors and the wave sums of an earlier group of
  // the same solve are still in red and fac (the same values)
  if (!reuse) {
    double r = INFINITY;
    for (int j = tid; j < n; j += NT) {
      const double* pj = d.partials + (size_t)j * kPartStride(T);
      if (pj[1] > 0.0) r = fmin(r, pj[0]);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) r = fmin(r, __shfl_xor(r, m, 64));
    if (lane == 0) red[wave] = r;
  }
  __syncthreads();
  double rho = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) rho = fmin(rho, red[w]);
  // tile factors, and eta, eta2 by a fixed tree over the VT threads
#pragma unroll
  for (int rr = 0; rr < (reuse ? 0 : R); ++rr) {
    const int v = tid + rr * NT;
    double e = 0.0, e2 = 0.0;
    for (int j = v; j < n; j += VT) {
      const double* pj = d.partials + (size_t)j * kPartStride(T);
      const double f = (pj[1] > 0.0 && isfinite(rho)) ? exp(-(pj[0] - rho) * d.inv_lambda) : 0.0;
      fac[j] = f;
      e += pj[1] * f;
      e2 += pj[2] * f * f;
    }
    e = wave_sum(e);
    e2 = wave_sum(e2);
    if (lane == 0) {
      red[NW + (v >> 6)] = e;
      red[2 * NW + (v >> 6)] = e2;
    }
  }
  __syncthreads();
  double eta = 0.0, eta2 = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    eta += red[NW + w];
    eta2 += red[2 * NW + w];
  }
  const bool ok = isfinite(rho) && eta > 0.0;
  double* res = d.result;
  // the slice of U*: partial sums over C tile ranges, each in tile order
  if (ok) {
    if constexpr (R == 1) {
      if (tid < C * L) {
        double sacc = 0.0;
        if (item) {
#pragma unroll
          for (int q = 0; q < kPre; ++q)
            if (j0 + q < j1) sacc = fma(sv[q], fac[j0 + q], sacc);
#pragma unroll 8
          for (int j = j0 + kPre; j < j1; ++j) sacc = fma(d.partials[(size_t)j * kPartStride(T) + 4 + o], fac[j], sacc);
        }
        part[tid] = sacc;
      }
    } else {
      for (int v = tid; v < C * L; v += NT) {
        const int vg = v / L, vo = u0 + (v - vg * L);
        const int a = vg * n / C, b = (vg + 1) * n / C;
        double sacc = 0.0;
        if (vo < u1) {
          // up to eight reads in flight, the products in tile order
          for (int j = a; j < b; j += 8) {
            double x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = j + q < b ? d.partials[(size_t)(j + q) * kPartStride(T) + 4 + vo] : 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q)
              if (j + q < b) sacc = fma(x[q], fac[j + q], sacc);
          }
        }
        part[v] = sacc;
      }
    }
  }
  __syncthreads();
  for (int i = u0 + tid; i < u1; i += NT) {
    const int t = i >> 2, ch = i & 3;
    double U;
    if (ok) {
      double sacc = part[i - u0];
      for (int rg = 1; rg < C; ++rg) sacc += part[rg * L + (i - u0)];
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
  if (d.wn || d.J_copy)
    for (int k = kb + tid; k < ke; k += NT) {
      const float J = (R == 1 && k == kb + tid) ? J0 : d.J[k];
      if (d.wn) d.wn[k] = (ok && isfinite(J)) ? exp(-((double)J - rho) * d.inv_lambda) / eta : 0.0;
      if (d.J_copy) d.J_copy[k] = J;
    }
  if (c == 0 && tid == 0) {
    const uint32_t tick = d.tick_fixed == 0xFFFFFFFFu ? *d.tick_slot : d.tick_fixed;
    double* rr = res + 4 * T;
    rr[RES_TICK] = (double)tick;
    if (ok) {
      const double jmin = rho + d.C0;
      rr[RES_STATUS] = 0.0;
      rr[RES_JMIN] = jmin;
      rr[RES_LOGETA] = log(eta) - jmin * d.inv_lambda;
      rr[RES_ESS] = eta * eta / eta2;
      rr[RES_ETA] = eta;
    } else {
      rr[RES_STATUS] = -5.0;
      rr[RES_JMIN] = NAN;
      rr[RES_LOGETA] = NAN;
      rr[RES_ESS] = 0.0;
      rr[RES_ETA] = 0.0;
    }
    if (d.tick_slot) *d.tick_slot = tick + 1u;
  }
}

__global__ __launch_bounds__(kMergeThreads) void k_fused_merge(FusedBatch batch) {
  extern __shared__ __align__(16) char lds[];
  const SolveDesc& d = batch.descs[blockIdx.x];
  if ((int)blockIdx.y >= merge_groups(d.T)) return;
  double* red = (double*)lds;
  merge_group<kMergeThreads>(d, blockIdx.y, red, red + 3 * (kMergeThreads / 64) + kMergeThreads);
}

// ------------------------------------------------------- served ring kernel
//
// Persistent kernel of the served path (see ring.hpp for the protocol): one
// workgroup per compute unit claims ring items in publication order.  A
// prep item copies a solve's upload block from pinned host memory into its
// device block and folds the latent block of every gate; a tile item runs
// one tile exactly as k_fused does; the workgroup that counts a solve's last
// tile merges its partials exactly as k_fused_merge does (the same function,
// the same summation order) and publishes the solve's completion.  Results,
// weights and the cost copy go to pinned host memory named in the
// descriptor, so the host reads them without a copy.

// Extra LDS of the served kernel beyond the fused layout: the merge's
// reductions and partial sums (its tile factors use the layout's fac table).
constexpr size_t kServedMergeBytes = sizeof(double) * (3 * (kMergeThreads / 64) + kMergeThreads);

// Host words are read with relaxed system-scope loads (coherent reads of
// host memory); device words are polled with relaxed agent-scope loads.
// Polling never fences: an acquire or release fence at agent or system scope
// writes back or invalidates a whole L2 on this GPU, so fences stand only
// where data changes hands (a tile's block, its partials, a solve's result).
__device__ __forceinline__ uint64_t ring_host_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ RingItem ring_host_item(const RingItem* p) {
  const uint64_t* q = (const uint64_t*)p;
  const uint64_t w0 = ring_host_load(q), w1 = ring_host_load(q + 1), w2 = ring_host_load(q + 2),
                 w3 = ring_host_load(q + 3);
  RingItem it;
  it.block = w0;
  it.src = w1;
  it.slot = (uint32_t)w2;
  it.k0 = (int32_t)(uint32_t)(w2 >> 32);
  it.count = (uint32_t)w3;
  it.seq = (uint32_t)(w3 >> 32);
  return it;
}

// Device copies of the host's tails, refreshed by one thread
// at a time (token) and at most once per refresh_ticks over the whole grid.
__device__ __forceinline__ void ring_refresh(const RingArgs& r) {
  const uint64_t now = __builtin_amdgcn_s_memrealtime();
  if (now - __hip_atomic_load(r.poll_time, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < r.refresh_ticks) return;
  uint32_t free_token = 0u;
  if (!__hip_atomic_compare_exchange_strong(r.poll, &free_token, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT))
    return;
  const uint64_t pt = ring_host_load(r.ptail);
  const uint64_t t = ring_host_load(r.tail);
  __hip_atomic_fetch_max(r.dptail, pt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_max(r.dtail, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(r.poll_time, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(r.poll, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Claim the next item of a queue (one thread) up to the device copy of its
// tail: the head is advanced by compare-and-swap; the item is read (from
// host memory, after the tail that covers it) before the claim: an item not
// yet claimed is never rewritten by the host, so what was read is the item
// the claim takes.
__device__ __forceinline__ bool ring_claim(const RingItem* items, uint32_t cap, uint64_t* head,
                                           const uint64_t* dtail, RingItem& it) {
  uint64_t hd = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t t = __hip_atomic_load(dtail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  while (hd < t) {
    it = ring_host_item(items + hd % cap);
    if (__hip_atomic_compare_exchange_strong(head, &hd, hd + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return true;
  }
  return false;
}

__device__ __forceinline__ void ring_put(int* m, const RingItem& it) {
  m[0] = (int)(uint32_t)it.block;
  m[1] = (int)(uint32_t)(it.block >> 32);
  m[2] = (int)(uint32_t)it.src;
  m[3] = (int)(uint32_t)(it.src >> 32);
  m[4] = (int)it.slot;
  m[5] = it.k0;
  m[6] = (int)it.count;
  m[7] = (int)it.seq;
}

__device__ __forceinline__ RingItem ring_get(const int* m) {
  RingItem it;
  it.block = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(m[0]) |
             ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(m[1]) << 32);
  it.src = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(m[2]) |
           ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(m[3]) << 32);
  it.slot = (uint32_t)__builtin_amdgcn_readfirstlane(m[4]);
  it.k0 = __builtin_amdgcn_readfirstlane(m[5]);
  it.count = (uint32_t)__builtin_amdgcn_readfirstlane(m[6]);
  it.seq = (uint32_t)__builtin_amdgcn_readfirstlane(m[7]);
  return it;
}

// Output m of gate g of the latent fold, formed exactly as fold_gate forms
// it (the same products in the same order), sixteen weight reads in flight.
__device__ __forceinline__ void fold_one(const SolveDesc& d, int g, int m, const DeviceWeights& w) {
  const int H = d.H;
  float* cache = d.cf_cache ? d.cf_cache + (size_t)g * H : nullptr;
  if ((d.fold_cached >> g) & 1u) {
    d.cfold[g * H + m] = cache[m];
    return;
  }
  const float* z = d.z + g * kLatent;
  double acc = w.b0[m];
#pragma unroll
  for (int j0 = 0; j0 < kLatent; j0 += 16) {
    double wv[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) wv[j] = w.w0lat[(size_t)(j0 + j) * H + m];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc = fma(wv[j], (double)z[j0 + j], acc);
  }
  d.cfold[g * H + m] = (float)acc;
  if (cache) cache[m] = (float)acc;
}

// A prep item, on the whole workgroup: the host's mirror into the device
// block, the folds (every gate at once over the workgroup), then the slot's
// ready word.
__device__ __forceinline__ void ring_prep(const RingArgs& ring, const RingItem& it, const DeviceWeights& w) {
  const int tid = threadIdx.x;
  const uint64_t* from = (const uint64_t*)it.src;
  uint64_t* to = (uint64_t*)(ring.pool + it.block);
  for (uint32_t i = tid; i < it.count / 8; i += kThreads) to[i] = ring_host_load(from + i);
  __syncthreads();   // the workgroup reads its own stores back (one L1)
  const SolveDesc& d = *(const SolveDesc*)(ring.pool + it.block);
  if (d.sdf_kind == 0)
    for (int i = tid; i < d.G * d.H; i += kThreads) fold_one(d, i / d.H, i % d.H, w);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the block, for tiles anywhere on the device
  __syncthreads();
  if (tid == 0) __hip_atomic_store(ring.prep + it.slot, it.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The merge of a solve on one workgroup, group after group.
__device__ __forceinline__ void ring_merge(const SolveDesc& d, double* scratch, double* fac) {
  const int ng = merge_groups(d.T);
  for (int c = 0; c < ng; ++c) {
    merge_group<kThreads>(d, c, scratch, fac, c > 0);
    __syncthreads();
  }
}

template <int P, int H, int NHH, bool PE>
__global__ __launch_bounds__(kThreads, 1) void k_served(RingArgs ring, DeviceWeights w, int Tm, int Gm,
                                                         int max_tiles) {
  constexpr int WPL = kWaves / NHH;
  constexpr int MB = H / WPL / 16;
  extern __shared__ __align__(16) char lds[];
  const Views V = make_views<P, H, NHH>(lds, Tm, Gm, max_tiles, PE ? w.feat_k32 : 0);
  double* mscratch = (double*)(lds + fused_lds<P, H, NHH>(Tm, Gm, max_tiles, PE ? w.feat_k32 : 0).total);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 4, nl = lane & 15;
  const int own = wave / WPL, gw = wave % WPL;
  FragT<P> wreg[MB][H / 32];
  const float scale_own = fused_setup<P, H, NHH, PE, MB>(V, w, tid, lane, own, gw, wreg);

  uint64_t ticket = ~0ull;   // thread 0: the tile-queue index this workgroup holds
  while (true) {
    __syncthreads();
    if (tid == 0) {
      // a queued prep item first; else the item of this workgroup's ticket,
      // once published (an exit item, or no item for wait_polls polls:
      // leave)
      int got = 0;
      RingItem item{};
      for (uint32_t n = 0;;) {
        ring_refresh(ring);
        if (ring_claim(ring.pitems, ring.pcap, ring.phead, ring.dptail, item)) {
          got = 1;
          break;
        }
        if (ticket == ~0ull) ticket = __hip_atomic_fetch_add(ring.head, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ticket < __hip_atomic_load(ring.dtail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
          item = ring_host_item(ring.items + ticket % ring.cap);
          ticket = ~0ull;
          got = item.k0 != kRingExit;
          break;
        }
        if (++n > ring.wait_polls) {
          __hip_atomic_store(ring.lost, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
      V.misc[0] = got;
      if (got) ring_put(V.misc + 1, item);
    }
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(V.misc[0])) break;
    const RingItem it = ring_get(V.misc + 1);
    if (it.k0 < 0) {
      ring_prep(ring, it, w);
      continue;
    }
    const uint32_t slot = it.slot, seq = it.seq, count = it.count;
    const SolveDesc& d = *(const SolveDesc*)(ring.pool + it.block);

    // tile: wait until the solve's block is ready, running queued prep items
    // meanwhile (state 1 ready, 2 a prep item to run, 3 gave up, 0 wait)
    int st = 0;
    for (uint32_t n = 0;;) {
      __syncthreads();
      if (tid == 0) {
        RingItem pi{};
        int s0 = 0;
        if (__hip_atomic_load(ring.prep + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == seq) {
          s0 = 1;
        } else {
          ring_refresh(ring);
          if (ring_claim(ring.pitems, ring.pcap, ring.phead, ring.dptail, pi)) {
            s0 = 2;
            ring_put(V.misc + 1, pi);
          } else if (++n > ring.wait_polls) {
            s0 = 3;
          } else {
            __builtin_amdgcn_s_sleep(4);
          }
        }
        V.misc[9] = s0;
      }
      __syncthreads();
      st = __builtin_amdgcn_readfirstlane(V.misc[9]);
      if (st == 1 || st == 3) break;
      if (st == 2) ring_prep(ring, ring_get(V.misc + 1), w);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool ok = st == 1;
    if (ok) fused_tile<P, H, NHH, PE, MB>(V, d, w, it.k0, wave, lane, gw, h, nl, scale_own, wreg);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
      if (!ok) __hip_atomic_store(ring.fail + slot, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      V.misc[10] = (int)__hip_atomic_fetch_add(ring.tiles + slot, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if ((uint32_t)__builtin_amdgcn_readfirstlane(V.misc[10]) + 1u != count) continue;
    // the solve's last tile: merge, then publish the completion
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool failed = __hip_atomic_load(ring.fail + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    if (!failed) ring_merge(d, mscratch, V.fac);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");   // the result in host memory, the warm start
    __syncthreads();
    if (tid == 0) {
      __hip_atomic_store(ring.tiles + slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ring.fail + slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ring.done + slot, failed ? (seq | kRingFailBit) : seq, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// ------------------------------------------------------- wide decoder (H = 512)
//
// At H = 512 a hidden layer's bfloat16 weights (512 KB) no longer fit in a
// compute unit, so the decoder streams them: the weights of one K-step of
// 32 inputs for all H neurons (one "slice", 32 KB in bfloat16, 16 KB in FP8)
// pass from L2 through a two-slice LDS ring, one slice per step with one
// workgroup barrier per step, while the query rows stay in registers through
// every layer.  Eight waves, two per SIMD: a pair of waves shares a block of
// 16 rows, each owning the neuron blocks of one parity (nb = 2 m + par), so a
// wave keeps 16 x 256 FP32 accumulators per layer (64 registers).  The
// weights are packed with their input index permuted so that the 8 operand
// slots of K-step ks are the values of neuron blocks 2 ks (slots 0-3) and
// 2 ks + 1 (slots 4-7) as one lane holds them in its accumulators (the
// product is the same sum in another order): each wave of a pair forms its
// half of the next K-step's operand from its own accumulators (or, for the
// first hidden layer, from layer 1 at the row's gate-frame point) and the
// two halves meet in a small LDS exchange buffer.  The two waves on a SIMD
// run each step in opposite order (vector work first / products first) so
// that one's vector work issues beside the other's matrix-core products.

constexpr int kWideWaves = 8;
constexpr int kWideThreads = 64 * kWideWaves;
constexpr int kWidePairs = kWideWaves / 2;      // row blocks of 16 per pass
// Owned neuron blocks per scheduling region of a K-step (fragment read-ahead
// depth): 2, 4 or 8, a template parameter of the kernel chosen per shape
// (see launch_fused).
constexpr int kWideRegionDefault = 4;

template <int P> __host__ __device__ constexpr int frag_bytes() { return PrecTraits<P>::fp8 ? 8 : 16; }

// Bytes of one weight slice: H / 16 fragments of 64 lanes.
template <int P, int H> __host__ __device__ constexpr int wide_slice_bytes() { return (H / 16) * 64 * frag_bytes<P>(); }

// Row stride of the folded latent table: the pad puts the gates' rows on
// different LDS banks (rows of one block read up to 8 gates at once).
template <int H> __host__ __device__ constexpr int wide_cf_stride() { return H + 4; }

// Input neuron of operand slot j (< 8) of lane group hq (= lane / 16) in
// K-step ks: the lane's accumulator values of blocks 2 ks and 2 ks + 1.
__host__ __device__ constexpr int wide_input(int ks, int hq, int j) {
  return 32 * ks + (j < 4 ? 4 * hq + j : 16 + 4 * hq + (j - 4));
}

// Operand exchange buffer: per pair, per step parity, per split term, per
// lane one operand (16 bytes bfloat16, 8 bytes FP8).
template <int P> __host__ __device__ constexpr int wide_xterm_bytes() { return 64 * frag_bytes<P>(); }
template <int P> __host__ __device__ constexpr int wide_xbuf_bytes() {
  return kWidePairs * 2 * PrecTraits<P>::splits * wide_xterm_bytes<P>();
}

template <int P, int H, int NHH>
__host__ __device__ FusedLds wide_lds(int Tm, int Gm, int max_tiles) {
  FusedLds L{};
  size_t o = 0;
  auto take = [&](size_t b) { const size_t r = o; o = (o + b + 15) / 16 * 16; return r; };
  L.act = take(2 * (size_t)wide_slice_bytes<P, H>());     // weight slice ring
  L.xch = take(wide_xbuf_bytes<P>());
  L.opart = take(sizeof(float) * kWidePairs * 2 * kRows);
  L.w1p = take(sizeof(float) * 4 * H);
  L.hb = take(sizeof(float) * NHH * H);
  L.wo = take(sizeof(float) * H);
  L.jl = take(sizeof(float) * 2 * kTileR);
  L.wt = take(sizeof(double) * (kTileR + 4));
  L.misc = take(64);
  L.rot = take(sizeof(float) * 8 * kTileR);
  L.pts = take(sizeof(float) * 4 * kTileR * Tm);          // control samples
  L.cf = take(sizeof(float) * Gm * wide_cf_stride<H>());
  L.rt = take(sizeof(float) * 9 * Gm);
  L.base = take(sizeof(float) * 3 * Gm * (Tm + 1));
  L.los = take(sizeof(float) * 2 * Tm);
  L.dp = take(sizeof(float) * 3 * kTileR * (Tm + 1));
  L.field = take(sizeof(float) * kTileR * Tm);
  L.fac = take(sizeof(double) * max_tiles);
  L.total = o;
  return L;
}

template <int P, int H, int NHH>
__device__ __forceinline__ Views make_wide_views(char* lds, int Tm, int Gm, int max_tiles) {
  const FusedLds L = wide_lds<P, H, NHH>(Tm, Gm, max_tiles);
  Views v{};
  v.act = lds + L.act;
  v.xch = lds + L.xch;
  v.samp = (float*)(lds + L.pts);
  v.opart = (float*)(lds + L.opart);
  v.w1p = (float*)(lds + L.w1p);
  v.hb = (float*)(lds + L.hb);
  v.wo = (float*)(lds + L.wo);
  v.cf = (float*)(lds + L.cf);
  v.rt = (float*)(lds + L.rt);
  v.base = (float*)(lds + L.base);
  v.los = (float*)(lds + L.los);
  v.dp = (float*)(lds + L.dp);
  v.field = (float*)(lds + L.field);
  v.jl = (float*)(lds + L.jl);
  v.wt = (double*)(lds + L.wt);
  v.fac = (double*)(lds + L.fac);
  v.misc = (int*)(lds + L.misc);
  v.rot = (float*)(lds + L.rot);
  return v;
}

// One slice's share of this thread (16-byte pieces, coalesced), held in
// native vector registers (a copy through HIP's uint4 struct becomes a
// memcpy that stays in scratch memory).
using u32x4 = __attribute__((ext_vector_type(4))) unsigned int;
template <int P, int H>
struct SliceCopy {
  static constexpr int N = wide_slice_bytes<P, H>() / 16 / kWideThreads;
  static_assert(N * 16 * kWideThreads == wide_slice_bytes<P, H>(), "slice split");
  u32x4 r[N];
  // g: the slice's first piece (wave-uniform).  It passes through an empty
  // asm so the compiler forms each step's addresses in place instead of
  // keeping every unrolled step's 64-bit addresses live in registers.
  __device__ __forceinline__ void load(const u32x4* g, int tid) {
    asm volatile("" : "+s"(g));
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = g[tid + i * kWideThreads];
  }
  __device__ __forceinline__ void store(u32x4* l, int tid) const {
#pragma unroll
    for (int i = 0; i < N; ++i) l[tid + i * kWideThreads] = r[i];
  }
};

// This wave's half (slots 4 par .. 4 par + 3) of one K-step's operand from
// its 4 activation values, into the exchange buffer x (the pair's buffer of
// the step's parity): bfloat16 splits a = hi (+ mid (+ lo)), two words per
// term; FP8 one word.
template <int P>
__device__ __forceinline__ void wide_put_half(char* x, int lane, int par, float (&v)[4], float inv) {
  using PT = PrecTraits<P>;
  if constexpr (PT::fp8) {
    float q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = fminf(v[i] * inv, 448.0f);
    uint32_t w = __builtin_amdgcn_cvt_pk_fp8_f32(q[0], q[1], 0u, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(q[2], q[3], w, true);
    *(uint32_t*)(x + lane * 8 + 4 * par) = w;
  } else if constexpr (PT::f16) {
    uint32_t h[2], l[2];
    split_f16(v, h, l);
    *(uint2*)(x + lane * 16 + 8 * par) = make_uint2(h[0], h[1]);
    *(uint2*)(x + wide_xterm_bytes<P>() + lane * 16 + 8 * par) = make_uint2(l[0], l[1]);
  } else {
#pragma unroll
    for (int sp = 0; sp < PT::splits; ++sp) {
      const uint32_t w0 = pack_bf16(v[0], v[1]), w1 = pack_bf16(v[2], v[3]);
      *(uint2*)(x + sp * wide_xterm_bytes<P>() + lane * 16 + 8 * par) = make_uint2(w0, w1);
      if (sp + 1 < PT::splits) {
        v[0] -= bf16_lo(w0);
        v[1] -= bf16_hi(w0);
        v[2] -= bf16_lo(w1);
        v[3] -= bf16_hi(w1);
      }
    }
  }
}

// Half operand of K-step ks of the first hidden layer: layer 1 (softplus of
// the point's product with W1[:, 0..2] plus the folded latent term of the
// row's gate) at neurons 32 ks + 16 par + 4 hq + i.
template <int P, int H>
__device__ __forceinline__ void wide_l1_half(const Views& V, const float (&pt)[4], int ks, int hq, int par, int lane,
                                             float inv, char* x) {
  const int n0 = 32 * ks + 16 * par + 4 * hq;
  const float4 c = *(const float4*)(V.cf + (int)pt[3] * wide_cf_stride<H>() + n0);
  const float cc[4] = {c.x, c.y, c.z, c.w};
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float4 w = *(const float4*)(V.w1p + 4 * (n0 + i));
    v[i] = softplus_act<P>(fmaf(w.x, pt[0], fmaf(w.y, pt[1], fmaf(w.z, pt[2], cc[i]))));
  }
  wide_put_half<P>(x, lane, par, v, inv);
}

// Half operand of K-step ks of the next hidden layer from this wave's
// accumulator block m = ks (neurons 32 ks + 16 par + 4 hq + i); FP8 scales
// and adds the bias here, F16X2 scales (its accumulators start at the scaled
// bias), the bfloat16 kinds start the accumulators at the bias.
template <int P>
__device__ __forceinline__ void wide_epi_half(const f32x4& acc, const float* hb, float scale, int ks, int hq, int par,
                                              int lane, float inv, char* x) {
  float v[4];
  float4 bb = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if constexpr (PrecTraits<P>::fp8) bb = *(const float4*)(hb + 32 * ks + 16 * par + 4 * hq);
  const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = softplus_act<P>(pre_act<P>(acc[i], scale, bv[i]));
  wide_put_half<P>(x, lane, par, v, inv);
}

// One K-step of one wave: acc[m] += W(slice)[2 m + par] x operand for its
// H / 32 neuron blocks, in regions of RG blocks that read the next
// region's weight fragments ahead; the first region also issues the global
// reads of the next slice, the last one its LDS stores.  prep() forms this
// wave's half of the next K-step's operand: before the products when VFIRST,
// after them otherwise.
template <int P, int H, bool VFIRST, int RG, class Prep>
__device__ __forceinline__ void wide_step(const char* slice, const char* xin, int lane, int par, f32x4 (&acc)[H / 32],
                                          Prep&& prep, SliceCopy<P, H>& pf, const u32x4* gsrc, u32x4* ldst, int tid) {
  using PT = PrecTraits<P>;
  constexpr int NS = PT::splits;
  constexpr int GR = RG, NG = H / 32 / GR;
  BFragT<P> bf[NS];
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) {
    if constexpr (PT::fp8) bf[sp] = *(const long*)(xin + lane * 8);
    else bf[sp] = __builtin_bit_cast(BFragT<P>, *(const uint4*)(xin + sp * wide_xterm_bytes<P>() + lane * 16));
  }
  if constexpr (VFIRST) {
    prep();
    sched_fence();
  }
  pf.load(gsrc, tid);
  const char* fb = slice + (size_t)(par * 64 + lane) * frag_bytes<P>();   // fragment 2 m + par at m * 128 lanes
  FragT<P> a[2][GR];
  auto fetch = [&](int g) {
#pragma unroll
    for (int i = 0; i < GR; ++i) a[g & 1][i] = *(const FragT<P>*)(fb + (size_t)(g * GR + i) * 128 * frag_bytes<P>());
  };
  fetch(0);
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (g + 1 < NG) fetch(g + 1);
    if (g == NG - 1) pf.store(ldst, tid);
#pragma unroll
    for (int sp = 0; sp < NS; ++sp)
#pragma unroll
      for (int i = 0; i < GR; ++i) {
        f32x4& c = acc[g * GR + i];
        c = mfma_lp<P>(a[g & 1][i], bf[sp], c);
      }
    sched_fence();
  }
  if constexpr (!VFIRST) prep();
}

template <int P, int H>
__device__ __forceinline__ void wide_acc_init(const float* hb, int hq, int par, f32x4 (&acc)[H / 32]) {
#pragma unroll
  for (int m = 0; m < H / 32; ++m) {
    if constexpr (PrecTraits<P>::fp8) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    else acc[m] = *(const f32x4*)(hb + 16 * (2 * m + par) + 4 * hq);
  }
}

// This wave's share of the output of its row block: softplus of the last
// hidden layer's owned neurons, dot with the output weights, summed over the
// row's 4 lane groups, into the pair's partial table.
template <int P, int H>
__device__ __forceinline__ void wide_output_part(const Views& V, const f32x4 (&acc)[H / 32], const float* hb,
                                                 float scale, int hq, int par, int lane, float* op_out) {
  float op = 0.0f;
#pragma unroll
  for (int m = 0; m < H / 32; ++m) {
    const int n0 = 16 * (2 * m + par) + 4 * hq;
    const float4 o4 = *(const float4*)(V.wo + n0);
    float4 bb = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if constexpr (PrecTraits<P>::fp8) bb = *(const float4*)(hb + n0);
    const float ow[4] = {o4.x, o4.y, o4.z, o4.w}, bv[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) op = fmaf(ow[i], softplus_fast(pre_act<P>(acc[m][i], scale, bv[i])), op);
  }
  op += __shfl_xor(op, 16, 64);
  op += __shfl_xor(op, 32, 64);
  if (lane < kRows) op_out[par * kRows + lane] = op;
}

// Output of row block c from the pair's two partials: max over each
// position's gates into the tile's field table (lanes 0 .. 15).
__device__ __forceinline__ void wide_output_rows(const Views& V, const EdgeConsts& e, const float* op_in, int c,
                                                 int lane) {
  const int row = lane & (kRows - 1);
  const float sv = op_in[row] + op_in[kRows + row] + e.bout;
  const int base = e.p * e.G;
  float best = sv;
  for (int g = 1; g < e.G; ++g) {
    const float o = __shfl(sv, base + g, 64);
    if (base + g < kRows) best = fmaxf(best, o);
  }
  const int q = c * e.Pc + e.p;
  if (lane < kRows && e.g == 0 && e.p < e.Pc && q < e.npos) V.field[q] = best;
}

template <int P, int H, int NHH, bool VFIRST, int RG>
__device__ __forceinline__ void wide_tile(const Views& V, const DeviceWeights& w, const SolveDesc& d, int npos,
                                          int wave, int lane, int tid) {
  using PT = PrecTraits<P>;
  constexpr int KS = H / 32;
  constexpr int SB = wide_slice_bytes<P, H>();
  constexpr int SPP = NHH * KS;                 // steps (slices) per pass
  constexpr int XB = PT::splits * wide_xterm_bytes<P>();
  const int hq = lane >> 4, nl = lane & 15;
  const int rb = wave >> 1, par = wave & 1;
  const u32x4* gw = (const u32x4*)w.hidden_lp;
  u32x4* ring = (u32x4*)V.act;
  char* xb = V.xch + rb * 2 * XB;                    // this pair's two exchange buffers
  float* opp = V.opart + rb * 2 * kRows;
  const float inv1 = PT::fp8 ? w.a_inv[0] : 1.0f;
  const float invB = (PT::fp8 && NHH == 2) ? w.a_inv[NHH - 1] : 1.0f;
  const float sA = PT::scaled ? w.w_scale[0] * w.a_scale[0] : 1.0f;
  const float sB = PT::scaled ? w.w_scale[NHH - 1] * w.a_scale[NHH - 1] : 1.0f;
  const int nblk = (npos + kRows / d.G - 1) / (kRows / d.G);
  const int npass = (nblk + kWidePairs - 1) / kWidePairs;
  const EdgeConsts ec = edge_consts(d, nl, npos, w.bout);
  // slice 0 and the first operand of pass 0
  for (int i = tid; i < SB / 16; i += kWideThreads) ring[i] = gw[i];
  alignas(16) float pt[4];
  chunk_point(V, ec, rb, pt);
  wide_l1_half<P, H>(V, pt, 0, hq, par, lane, inv1, xb);
  __syncthreads();
  for (int j = 0; j < npass; ++j) {
    const int c = j * kWidePairs + rb;
    // ---- first hidden layer
    f32x4 accA[H / 32];
    wide_acc_init<P, H>(V.hb, hq, par, accA);
    for (int ks = 0; ks < KS; ++ks) {
      const int nxt = ks + 1 < SPP ? ks + 1 : 0;
      SliceCopy<P, H> pf;
      wide_step<P, H, VFIRST, RG>(V.act + (ks & 1) * SB, xb + (ks & 1) * XB, lane, par, accA, [&]() {
        if (ks + 1 < KS) {
          wide_l1_half<P, H>(V, pt, ks + 1, hq, par, lane, inv1, xb + ((ks + 1) & 1) * XB);
        } else if (NHH == 1) {
          // the first operand of the next pass (unused after the last)
          chunk_point(V, ec, c + kWidePairs, pt);
          wide_l1_half<P, H>(V, pt, 0, hq, par, lane, inv1, xb);
        }
      }, pf, gw + (size_t)nxt * (SB / 16), ring + ((ks + 1) & 1) * (SB / 16), tid);
      __syncthreads();
    }
    if constexpr (NHH == 2) {
      // ---- second hidden layer, its first operand from the final accA
      wide_epi_half<P>(accA[0], V.hb, sA, 0, hq, par, lane, invB, xb);
      __syncthreads();
      f32x4 accB[H / 32];
      wide_acc_init<P, H>(V.hb + H, hq, par, accB);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int nxt = KS + ks + 1 < SPP ? KS + ks + 1 : 0;
        SliceCopy<P, H> pf;
        wide_step<P, H, VFIRST, RG>(V.act + (ks & 1) * SB, xb + (ks & 1) * XB, lane, par, accB, [&]() {
          if (ks + 1 < KS) {
            wide_epi_half<P>(accA[ks + 1], V.hb, sA, ks + 1, hq, par, lane, invB, xb + ((ks + 1) & 1) * XB);
          } else {
            chunk_point(V, ec, c + kWidePairs, pt);
            wide_l1_half<P, H>(V, pt, 0, hq, par, lane, inv1, xb);
          }
        }, pf, gw + (size_t)nxt * (SB / 16), ring + ((ks + 1) & 1) * (SB / 16), tid);
        __syncthreads();
      }
      wide_output_part<P, H>(V, accB, V.hb + H, sB, hq, par, lane, opp);
    } else {
      wide_output_part<P, H>(V, accA, V.hb, sA, hq, par, lane, opp);
    }
    __syncthreads();
    if (par == 0) wide_output_rows(V, ec, opp, c, lane);
  }
}

template <int P, int H, int NHH, int RG>
__global__ __launch_bounds__(kWideThreads, 1) void k_wide(FusedBatch batch, DeviceWeights w, int Tm, int Gm,
                                                           int max_tiles) {
  extern __shared__ __align__(16) char lds[];
  const Views V = make_wide_views<P, H, NHH>(lds, Tm, Gm, max_tiles);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < 4 * H; i += kWideThreads) V.w1p[i] = w.w1p[i];
  for (int i = tid; i < NHH * H; i += kWideThreads) V.hb[i] = bias_start<P>(w.hbias[i], PrecTraits<P>::scaled ? w.w_scale[i / H] : 1.0f);
  for (int i = tid; i < H; i += kWideThreads) V.wo[i] = w.wout[i];
  while (true) {
    __syncthreads();
    if (tid == 0) V.misc[0] = (int)atomicAdd(batch.tile_counter, 1u);
    __syncthreads();
    // uniform across the workgroup: descriptor reads go to scalar registers
    const int tile = __builtin_amdgcn_readfirstlane(V.misc[0]);
    if (tile >= batch.n_tiles) break;
    const int2 tl0 = batch.tiles[tile];
    const int2 tl = make_int2(__builtin_amdgcn_readfirstlane(tl0.x), __builtin_amdgcn_readfirstlane(tl0.y));
    const SolveDesc& d = batch.descs[tl.x];
    const int k0 = tl.y;
    const int Re = min(kTileR, d.K - k0);
    const uint32_t tick = d.tick_fixed == 0xFFFFFFFFu ? *d.tick_slot : d.tick_fixed;
    tile_prologue(V, d, k0, Re, tick, H, wide_cf_stride<H>() - H);
    // waves w and w + 4 share a SIMD: one forms its operands before its
    // products, the other after
    if (wave < kWideWaves / 2) wide_tile<P, H, NHH, true, RG>(V, w, d, Re * d.T, wave, lane, tid);
    else wide_tile<P, H, NHH, false, RG>(V, w, d, Re * d.T, wave, lane, tid);
    __syncthreads();
    tile_epilogue(V, d, k0, Re, tick);
  }
}

// ------------------------------------------------------------------ host side

template <int P, int H, int NHH, bool PE>
static hipError_t launch_fused_t(const FusedBatch& b, const DeviceWeights& w, int Tm, int Gm,
                                 int max_tiles, hipStream_t s) {
  const FusedLds L = fused_lds<P, H, NHH>(Tm, Gm, max_tiles, PE ? w.feat_k32 : 0);
  {
    // raise the kernel's dynamic LDS limit to the largest size launched so far
    // (engines on several threads may launch the same instantiation)
    static std::mutex mu;
    static int max_set = 0;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)L.total > max_set) {
      hipError_t e = hipFuncSetAttribute((const void*)k_fused<P, H, NHH, PE>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
      if (e != hipSuccess) return e;
      max_set = (int)L.total;
    }
  }
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int grid = std::max(1, std::min(b.n_tiles, ncu));
  hipLaunchKernelGGL((k_fused<P, H, NHH, PE>), dim3(grid), dim3(kThreads), L.total, s, b, w, Tm,
                     Gm, max_tiles);
  return hipGetLastError();
}

template <int P, int H, int NHH, int RG>
static hipError_t launch_wide_t(const FusedBatch& b, const DeviceWeights& w, int Tm, int Gm,
                                int max_tiles, hipStream_t s) {
  const FusedLds L = wide_lds<P, H, NHH>(Tm, Gm, max_tiles);
  {
    static std::mutex mu;
    static int max_set = 0;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)L.total > max_set) {
      hipError_t e = hipFuncSetAttribute((const void*)k_wide<P, H, NHH, RG>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
      if (e != hipSuccess) return e;
      max_set = (int)L.total;
    }
  }
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int grid = std::max(1, std::min(b.n_tiles, ncu));
  hipLaunchKernelGGL((k_wide<P, H, NHH, RG>), dim3(grid), dim3(kWideThreads), L.total, s, b, w, Tm, Gm,
                     max_tiles);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_fused_p(const FusedBatch& b, const DeviceWeights& w, int Tm, int Gm, int mt,
                                 hipStream_t s, int rg) {
  const int nhh = w.n_hidden - 1;
  const bool pe = w.feat_ksteps > 0;
  if (w.H == 128 && nhh == 1) return pe ? launch_fused_t<P, 128, 1, true>(b, w, Tm, Gm, mt, s) : launch_fused_t<P, 128, 1, false>(b, w, Tm, Gm, mt, s);
  if (w.H == 128 && nhh == 2) return pe ? launch_fused_t<P, 128, 2, true>(b, w, Tm, Gm, mt, s) : launch_fused_t<P, 128, 2, false>(b, w, Tm, Gm, mt, s);
  if (w.H == 256 && nhh == 1) return pe ? launch_fused_t<P, 256, 1, true>(b, w, Tm, Gm, mt, s) : launch_fused_t<P, 256, 1, false>(b, w, Tm, Gm, mt, s);
  if (w.H == 256 && nhh == 2) return pe ? launch_fused_t<P, 256, 2, true>(b, w, Tm, Gm, mt, s) : launch_fused_t<P, 256, 2, false>(b, w, Tm, Gm, mt, s);
  if (pe) return hipErrorInvalidValue;   // the H = 512 decoder has no encoded-point layer 1
  if (w.H == 512) {
    if (rg != 2 && rg != 4 && rg != 8) return hipErrorInvalidValue;
    if (nhh == 1)
      return rg == 2 ? launch_wide_t<P, 512, 1, 2>(b, w, Tm, Gm, mt, s)
                     : rg == 4 ? launch_wide_t<P, 512, 1, 4>(b, w, Tm, Gm, mt, s) : launch_wide_t<P, 512, 1, 8>(b, w, Tm, Gm, mt, s);
    if (nhh == 2)
      return rg == 2 ? launch_wide_t<P, 512, 2, 2>(b, w, Tm, Gm, mt, s)
                     : rg == 4 ? launch_wide_t<P, 512, 2, 4>(b, w, Tm, Gm, mt, s) : launch_wide_t<P, 512, 2, 8>(b, w, Tm, Gm, mt, s);
  }
  return hipErrorInvalidValue;
}

// Zero the counter and fold (prep), then the decoder kernel of the precision.
static hipError_t launch_prep_decoder(const FusedBatch& b, int n_solves, const DeviceWeights& w, int max_T,
                                      int max_G, int max_tiles, hipStream_t s, hipEvent_t begin, hipEvent_t end,
                                      int wide_region) {
  hipLaunchKernelGGL(k_fused_prep, dim3(max_G, n_solves), dim3(256), 0, s, b, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (begin && (e = hipEventRecord(begin, s)) != hipSuccess) return e;
  switch (w.precision) {
    case P_BF16: e = launch_fused_p<P_BF16>(b, w, max_T, max_G, max_tiles, s, wide_region); break;
    case P_BF16X2: e = launch_fused_p<P_BF16X2>(b, w, max_T, max_G, max_tiles, s, wide_region); break;
    case P_BF16X3: e = launch_fused_p<P_BF16X3>(b, w, max_T, max_G, max_tiles, s, wide_region); break;
    case P_FP8: e = launch_fused_p<P_FP8>(b, w, max_T, max_G, max_tiles, s, wide_region); break;
    case P_F16X2: e = launch_fused_p<P_F16X2>(b, w, max_T, max_G, max_tiles, s, wide_region); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (end && (e = hipEventRecord(end, s)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_fused(const FusedBatch& b, int n_solves, const DeviceWeights& w, int max_T, int max_G,
                        int max_tiles, hipStream_t s, hipEvent_t begin, hipEvent_t end, int wide_region) {
  hipError_t e = launch_prep_decoder(b, n_solves, w, max_T, max_G, max_tiles, s, begin, end, wide_region);
  if (e != hipSuccess) return e;
  // per workgroup: the reductions, n tile factors, C x L <= kMergeThreads partial sums
  const size_t merge_lds = sizeof(double) * (3 * (kMergeThreads / 64) + (size_t)max_tiles + kMergeThreads);
  hipLaunchKernelGGL(k_fused_merge, dim3(n_solves, merge_groups(max_T)), dim3(kMergeThreads), merge_lds, s, b);
  return hipGetLastError();
}

template <int P, int H, int NHH, bool PE>
static hipError_t launch_served_t(const RingArgs& r, const DeviceWeights& w, int Tm, int Gm, int max_tiles,
                                  int grid, hipStream_t s) {
  const size_t bytes = fused_lds<P, H, NHH>(Tm, Gm, max_tiles, PE ? w.feat_k32 : 0).total + kServedMergeBytes;
  {
    static std::mutex mu;
    static int max_set = 0;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)bytes > max_set) {
      hipError_t e = hipFuncSetAttribute((const void*)k_served<P, H, NHH, PE>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e != hipSuccess) return e;
      max_set = (int)bytes;
    }
  }
  hipLaunchKernelGGL((k_served<P, H, NHH, PE>), dim3(grid), dim3(kThreads), bytes, s, r, w, Tm, Gm, max_tiles);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_served_p(const RingArgs& r, const DeviceWeights& w, int Tm, int Gm, int mt, int grid,
                                  hipStream_t s) {
  const int nhh = w.n_hidden - 1;
  const bool pe = w.feat_ksteps > 0;
  if (w.H == 128 && nhh == 1) return pe ? launch_served_t<P, 128, 1, true>(r, w, Tm, Gm, mt, grid, s) : launch_served_t<P, 128, 1, false>(r, w, Tm, Gm, mt, grid, s);
  if (w.H == 128 && nhh == 2) return pe ? launch_served_t<P, 128, 2, true>(r, w, Tm, Gm, mt, grid, s) : launch_served_t<P, 128, 2, false>(r, w, Tm, Gm, mt, grid, s);
  if (w.H == 256 && nhh == 1) return pe ? launch_served_t<P, 256, 1, true>(r, w, Tm, Gm, mt, grid, s) : launch_served_t<P, 256, 1, false>(r, w, Tm, Gm, mt, grid, s);
  if (w.H == 256 && nhh == 2) return pe ? launch_served_t<P, 256, 2, true>(r, w, Tm, Gm, mt, grid, s) : launch_served_t<P, 256, 2, false>(r, w, Tm, Gm, mt, grid, s);
  return hipErrorInvalidValue;
}

hipError_t launch_served(const RingArgs& r, const DeviceWeights& w, int max_T, int max_G, int max_tiles,
                         hipStream_t s) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int grid = std::max(1, ncu);
  switch (w.precision) {
    case P_BF16: return launch_served_p<P_BF16>(r, w, max_T, max_G, max_tiles, grid, s);
    case P_BF16X2: return launch_served_p<P_BF16X2>(r, w, max_T, max_G, max_tiles, grid, s);
    case P_BF16X3: return launch_served_p<P_BF16X3>(r, w, max_T, max_G, max_tiles, grid, s);
    case P_FP8: return launch_served_p<P_FP8>(r, w, max_T, max_G, max_tiles, grid, s);
    case P_F16X2: return launch_served_p<P_F16X2>(r, w, max_T, max_G, max_tiles, grid, s);
    default: return hipErrorInvalidValue;
  }
}

size_t served_lds_bytes(int precision, int H, int n_hidden, int Tm, int Gm, int max_tiles, int feat_ks) {
  if (H != 128 && H != 256) return 0;
  return fused_lds_bytes(precision, H, n_hidden, Tm, Gm, max_tiles, feat_ks) + kServedMergeBytes;
}

hipError_t tune_wide_region(const FusedBatch& b, int n_solves, const DeviceWeights& w, int max_T, int max_G,
                            int max_tiles, hipStream_t s, int* best) {
  *best = kWideRegionDefault;
  if (w.H != 512) return hipSuccess;
  int ncu = 0, dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  // the first tiles of the batch (longest first), two per compute unit
  FusedBatch part = b;
  part.n_tiles = std::min(b.n_tiles, 2 * ncu);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    hipEventDestroy(t0);
    return e;
  }
  float best_ms = INFINITY;
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep)
    for (const int rg : {2, 4, 8}) {
      e = launch_prep_decoder(part, n_solves, w, max_T, max_G, max_tiles, s, t0, t1, rg);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (e != hipSuccess) break;
      if (ms < best_ms) {
        best_ms = ms;
        *best = rg;
      }
    }
  hipEventDestroy(t0);
  hipEventDestroy(t1);
  return e;
}

int fused_tile_rollouts(int, int, int) { return kTileR; }

bool fused_supported(int precision, int H, int n_hidden) {
  if (!(precision == P_BF16 || precision == P_BF16X2 || precision == P_BF16X3 || precision == P_FP8 ||
        precision == P_F16X2))
    return false;
  return (H == 128 || H == 256 || H == 512) && (n_hidden == 2 || n_hidden == 3);
}

size_t fused_lds_bytes(int precision, int H, int n_hidden, int Tm, int Gm, int max_tiles, int feat_ks) {
  auto pick = [&](auto p_tag) -> size_t {
    constexpr int P = decltype(p_tag)::value;
    if (H == 512)
      return n_hidden == 2 ? wide_lds<P, 512, 1>(Tm, Gm, max_tiles).total : wide_lds<P, 512, 2>(Tm, Gm, max_tiles).total;
    if (n_hidden == 2)
      return H == 128 ? fused_lds<P, 128, 1>(Tm, Gm, max_tiles, feat_ks).total
                      : fused_lds<P, 256, 1>(Tm, Gm, max_tiles, feat_ks).total;
    return H == 128 ? fused_lds<P, 128, 2>(Tm, Gm, max_tiles, feat_ks).total
                    : fused_lds<P, 256, 2>(Tm, Gm, max_tiles, feat_ks).total;
  };
  switch (precision) {
    case P_BF16: return pick(std::integral_constant<int, P_BF16>{});
    case P_BF16X2: return pick(std::integral_constant<int, P_BF16X2>{});
    case P_BF16X3: return pick(std::integral_constant<int, P_BF16X3>{});
    case P_FP8: return pick(std::integral_constant<int, P_FP8>{});
    case P_F16X2: return pick(std::integral_constant<int, P_F16X2>{});
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

// IEEE half, round to nearest even (subnormals included; beyond 65504 rounds
// to the largest finite value, which the callers' scaling never reaches).
static uint16_t host_f16_rne(float x) {
  const uint16_t sign = std::signbit(x) ? 0x8000 : 0x0000;
  const double a = fabs((double)x);
  if (a < 0x1p-14) return sign | (uint16_t)nearbyint(a * 0x1p24);   // 1024 encodes 2^-14 itself
  int e;
  double m = frexp(a, &e);                // a = m 2^e, m in [0.5, 1)
  double q = nearbyint(m * 2048.0);       // 11 significant bits
  if (q == 2048.0) { q = 1024.0; ++e; }
  const int E = e - 1 + 15;
  if (E >= 31) return sign | 0x7BFF;
  return sign | (uint16_t)((E << 10) | ((int)q - 1024));
}

static float host_f16_to_float(uint16_t h) {
  const int e = (h >> 10) & 31, m = h & 1023;
  const double v = e == 0 ? ldexp((double)m, -24) : ldexp((double)(1024 + m), e - 25);
  return (float)((h & 0x8000) ? -v : v);
}

void pack_pe_weights_f16(int H, int n_feat, int ld, const float* W0, std::vector<uint8_t>& blob, float& scale) {
  const int K32 = (n_feat + 31) / 32;
  float amax = 0.0f;
  for (int m = 0; m < H; ++m)
    for (int f = 0; f < n_feat; ++f) amax = std::max(amax, fabsf(W0[(size_t)m * ld + f]));
  int e = 0;
  if (amax > 0.0f) frexpf(amax, &e);      // amax in [2^(e-1), 2^e): amax / scale < 2^15
  scale = amax > 0.0f ? ldexpf(1.0f, e - 15) : 1.0f;
  blob.assign((size_t)(H / 16) * K32 * 2 * 64 * 16, 0);
  for (int mb = 0; mb < H / 16; ++mb)
    for (int ks = 0; ks < K32; ++ks)
      for (int lane = 0; lane < 64; ++lane)
        for (int j = 0; j < 8; ++j) {
          const int m = 16 * mb + lane % 16, f = 32 * ks + 8 * (lane / 16) + j;
          const float v = f < n_feat ? W0[(size_t)m * ld + f] / scale : 0.0f;
          const uint16_t hi = host_f16_rne(v);
          const uint16_t lo = host_f16_rne(v - host_f16_to_float(hi));
          const size_t fi = (((size_t)mb * K32 + ks) * 2) * 64 + lane;
          memcpy(&blob[fi * 16 + 2 * j], &hi, 2);
          memcpy(&blob[(fi + 64) * 16 + 2 * j], &lo, 2);
        }
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
  const int NB = H / 16, KS = H / 32;
  const bool fp8 = precision == P_FP8, f16 = precision == P_F16X2;
  const size_t esz = fp8 ? 8 : 16;
  blob.assign((size_t)nhh * NB * KS * 64 * esz, 0);
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
    } else if (f16) {
      // power-of-two scale 2^-s with the largest bfloat16 weight times 2^s in
      // [2^14, 2^15): every bfloat16 weight within 2^-29 of the largest then
      // has an exact normal half image (8 significant bits of 11)
      float amax = 0.0f;
      for (size_t i = 0; i < (size_t)H * H; ++i) {
        const uint32_t hb = (uint32_t)host_bf16_rne(W[i]) << 16;
        float b;
        memcpy(&b, &hb, 4);
        amax = std::max(amax, fabsf(b));
      }
      if (!std::isfinite(amax)) return MPPI_EINVAL;
      int e = 0;
      if (amax > 0.0f) frexpf(amax, &e);    // amax in [2^(e-1), 2^e)
      scale = amax > 0.0f ? ldexpf(1.0f, e - 15) : 1.0f;
      w_scale[l] = scale;
    }
    // H <= 256: fragment (l, nb, ks, lane) at (((l NB + nb) KS + ks) 64 + lane),
    // as frag_index<H> lays it out, operand slot j = input 32 ks + 8 (lane / 16) + j.
    // H = 512: slices (l KS + ks) of NB fragments, ((l KS + ks) NB + nb) 64 + lane,
    // operand slot j = input wide_input(ks, lane / 16, j).
    const bool wide = H == 512;
    for (int nb = 0; nb < NB; ++nb)
      for (int ks = 0; ks < KS; ++ks)
        for (int lane = 0; lane < 64; ++lane) {
          const int m = 16 * nb + lane % 16;
          const size_t fi = wide ? (((size_t)l * KS + ks) * NB + nb) * 64 + lane
                                 : (((size_t)l * NB + nb) * KS + ks) * 64 + lane;
          for (int j = 0; j < 8; ++j) {
            const int k = wide ? wide_input(ks, lane / 16, j) : 32 * ks + 8 * (lane / 16) + j;
            const float v = W[(size_t)m * H + k];
            if (fp8) {
              blob[fi * 8 + j] = host_e4m3(v / scale);
            } else if (f16) {
              const uint32_t hb = (uint32_t)host_bf16_rne(v) << 16;
              float b;
              memcpy(&b, &hb, 4);
              const uint16_t h = host_f16_rne(b / scale);   // exact power-of-two scaling
              memcpy(&blob[fi * 16 + 2 * j], &h, 2);
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
