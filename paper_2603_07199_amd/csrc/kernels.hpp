// Host-side launchers of the device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "../../include/mppi.h"

#include "ring.hpp"
#include "solve_desc.hpp"
#include "weights.hpp"

namespace mppi {

struct PlainShape {
  int K, T, G, sdf_kind;
};

// Plain path: rollout -> SDF -> cost -> LSE -> weighted average for one solve
// whose descriptor is at device address dd.  The optional events bracket the
// SDF kernel (the dominant one).
hipError_t launch_plain(const SolveDesc* dd, const PlainShape& shape, const DeviceWeights& w,
                        hipStream_t s, hipEvent_t sdf_begin, hipEvent_t sdf_end);

// Latent fold c_g = W1[:, 3:] z_g + b1 for the gates of n_solves descriptors
// (the plain path; the fused path folds in its prep kernel).
hipError_t launch_fold(const SolveDesc* descs, int n_solves, int G_max, const DeviceWeights& w,
                       hipStream_t s);

// Fused path: one persistent launch over the tiles of a batch of solves.
struct FusedBatch {
  const SolveDesc* descs;    // device array of n_solves descriptors
  const int2* tiles;         // device array of (solve index, first rollout)
  int n_tiles;
  uint32_t* tile_counter;    // device work counter (zeroed by the launcher)
};

// n_solves descriptors, max_T / max_G over them, max_tiles = most tiles of
// one solve.  begin/end (optional) bracket the fused kernel itself.
// wide_region: the H = 512 decoder's neuron blocks per scheduling region
// (2, 4 or 8; ignored for H <= 256).
hipError_t launch_fused(const FusedBatch& b, int n_solves, const DeviceWeights& w, int max_T, int max_G,
                        int max_tiles, hipStream_t s, hipEvent_t begin, hipEvent_t end, int wide_region);

// Times the H = 512 decoder with each region size (2, 4, 8; twice each) on the
// batch's first tiles (two per compute unit; prep and decoder only, which
// write nothing but tile partials, costs and field values that the next full
// launch overwrites) and returns the fastest in *best.  Synchronous.  The
// region size changes only the order of independent matrix-core products,
// so every choice gives the same results bit for bit.
hipError_t tune_wide_region(const FusedBatch& b, int n_solves, const DeviceWeights& w, int max_T, int max_G,
                            int max_tiles, hipStream_t s, int* best);

// Served path: the persistent ring kernel (see ring.hpp), one workgroup per
// compute unit, for H <= 256; it runs until each workgroup has taken one of
// the exit items the host publishes (or, without the host, until a bounded
// wait gives up).  max_T,
// max_G, max_tiles: the largest solve the engine accepts (LDS layout).
hipError_t launch_served(const RingArgs& r, const DeviceWeights& w, int max_T, int max_G, int max_tiles,
                         hipStream_t s);
// LDS bytes of one served workgroup (0: no served kernel for this width).
size_t served_lds_bytes(int precision, int H, int n_hidden, int Tm, int Gm, int max_tiles, int feat_ks);

// Rollouts per fused tile for a precision / width (the unit of work of the
// persistent kernel).
int fused_tile_rollouts(int precision, int H, int G);

// Whether the fused kernel exists for this precision / width / depth, and the
// LDS bytes one workgroup needs for the given horizon, gate count and tiles.
bool fused_supported(int precision, int H, int n_hidden);
size_t fused_lds_bytes(int precision, int H, int n_hidden, int Tm, int Gm, int max_tiles, int feat_ks);
constexpr size_t kMaxLdsBytes = 160 * 1024;

// Quantise and pack the hidden H x H layers for a low-precision variant
// (BF16, BF16X2, FP8) in the fused kernel's operand order.  Returns an
// mppi_status.
// Encoded-point columns of layer 0 for the fused decoder (see DeviceWeights).
void pack_pe_weights_f16(int H, int n_feat, int ld, const float* W0, std::vector<uint8_t>& blob, float& scale);
int pack_lowp_weights(int precision, int H, int n_hidden, const mppi_sdf_weights* w,
                      std::vector<uint8_t>& blob, std::vector<float>& w_scale,
                      std::vector<float>& a_scale, std::vector<float>& a_inv);

// Library-owned device scratch of the entry point that allocates nothing
// (mppi_step_noalloc), one array per device for the life of the process.
constexpr size_t kScratchBytes = (size_t)MPPI_NOALLOC_SCRATCH_BYTES;
// Device address of the array on `device` (which the caller has made
// current), looked up once per device.
hipError_t scratch_device_address(int device, void** out);
// Serialises the calls that use the array of `device` within the process.
std::mutex& scratch_use_mutex(int device);

}  // namespace mppi
