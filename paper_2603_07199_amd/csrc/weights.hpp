// Device-resident decoder weights, packed once at engine creation.
//
// The first layer's coordinate columns (H x 3, padded to 4) and the output
// row stay float32 for the vector units; the first layer's latent block is
// folded per solve into a bias (W1[:, 3:] z + b1), an exact re-association of
// the concatenated input [p; z] of Section III-B.  Hidden H x H layers are
// packed in matrix-core operand order for the chosen precision.
#pragma once
#include <stdint.h>

namespace mppi {

struct DeviceWeights {
  int H, n_hidden, precision;
  const float* w1p;      // H x 4: W1[:, 0..2], 0
  const float* hbias;    // (n_hidden - 1) x H
  const float* wout;     // H
  const double* w0lat;   // 64 x H (transposed): latent block of the first layer (float32 values)
  const double* b0;      // H: first-layer bias
  float bout;
  // FP32: per hidden layer, fragments [mb][ks][64] of W[16 mb + lane%16][4 ks + lane/16]
  const float* hidden_f32;
  // BF16 family / FP8: per hidden layer, fragments [16-neuron block][K-step][64 lanes] (kernels_fused.hip)
  const void* hidden_lp;
  const float* w_scale;  // FP8: per hidden layer weight scale
  const float* a_scale;  // FP8: per hidden layer activation scale
  const float* a_inv;    // FP8: 1 / a_scale
  // positional encoding (pe_freqs > 0): n_feat = 3 + 6 pe_freqs features;
  // W1's feature columns as 16x16x4 FP32 operand fragments
  // [H/16][feat_ksteps][64] = W1[16 mb + lane % 16][4 ks + lane / 16] (0 past n_feat)
  int pe_freqs, n_feat, feat_ksteps;
  const float* w1pe;
  // the same columns for the fused decoder as FP16 16x16x32 A fragments of
  // W1 / w1pe_scale split into two terms, [H/16][feat_k32][2][64] x 8 halves
  // = term of W1[16 mb + lane % 16][32 ks + 8 (lane / 16) + j] (0 past n_feat)
  int feat_k32;
  float w1pe_scale;
  const void* w1pe16;
};

}  // namespace mppi
