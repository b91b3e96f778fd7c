// MPPI engine: the C ABI of include/mppi.h.
//
// Host work per solve (float64, then rounded once to float32):
//  - validation of the request;
//  - L = chol(Sigma) for delta u = L n (Section IV-A: delta u ~ N(0, Sigma));
//  - gate frames: R_g^T and the offsets of the local rollout frame, so that a
//    device position dp (relative to p0 + v0 t dt) maps into gate g's frame
//    as R_g^T dp + base_g(t) (Section IV-B-3: world points are mapped into the
//    cached gate/camera frame before the decoder is queried);
//  - the rollout-independent part of the progress cost (eq. 5), which cancels
//    in the weights (eq. mppi_update) and is added back to reported costs.
// Everything else, including the latent fold of the decoder's first layer,
// runs in the device kernels.
//
// Three ways to run solves share one staging routine and one launch routine:
//  - mppi_step: one blocking solve;
//  - mppi_submit / mppi_poll: a scheduler thread admits queued requests by
//    device-memory budget, batches what is admissible and launches each batch
//    on a free stream while earlier batches still run (continuous batching);
//  - mppi_batch_*: requests staged once into device memory and launched
//    repeatedly (fixed fleets, benchmarks): inputs stay resident in HBM.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/mppi.h"
#include "host_core.hpp"
#include "kernels.hpp"
#include "solve_desc.hpp"
#include "weights.hpp"

using namespace mppi;

namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

bool isfin(double x) { return std::isfinite(x); }

struct InstInfo {
  uint64_t id;
  int U_len;      // valid entries of the resident sequence
  bool busy;      // a served solve or a staged batch holds this instance
  // object permanence: the frame of each gate as last observed (its folded
  // latent is cached on the device, mppi_engine::instCf)
  uint32_t seen = 0;             // bit g: gate g observed at least once
  double R[kMaxG][9] = {};
  double t[kMaxG][3] = {};
};

// Deep copy of a request for the served path.
struct OwnedRequest {
  mppi_request req;
  std::vector<double> U;
  std::vector<float> z;
  std::vector<mppi_gate> gates;
  void take(const mppi_request& r, int latent) {
    req = r;
    if (r.U_nom) {
      U.assign(r.U_nom, r.U_nom + 4 * (size_t)r.T);
      req.U_nom = U.data();
    }
    const int G = r.G > 0 && r.gates ? r.G : 0;
    z.assign((size_t)G * latent, 0.0f);
    gates.assign(r.gates, r.gates + G);
    for (int g = 0; g < G; ++g) {
      // an unobserved gate (z == NULL) stays NULL
      if (r.gates[g].z) memcpy(&z[(size_t)g * latent], r.gates[g].z, sizeof(float) * latent);
      gates[g].z = r.gates[g].z ? &z[(size_t)g * latent] : nullptr;
    }
    req.gates = gates.data();
  }
};

// One solve living in device memory.
struct Solve {
  uint64_t ticket = 0;
  int K = 0, T = 0, G = 0;
  int slot = -1;
  uint32_t flags = 0;
  uint64_t off = 0, bytes = 0, footprint = 0;
  SolveLayout lay{};
  SolveDesc desc{};
  double C0 = 0.0;
  double v0[3] = {0, 0, 0};
  double dt = 0.0;
  bool exports = false, want_w = true, want_J = true;
  uint64_t t_submit = 0, t_admit = 0, t_done = 0;
  std::vector<double> res;   // 4T + RES_SCALARS
  std::vector<double> wn;    // K
  std::vector<float> J;      // K
  std::vector<float> samples, pos, sdf;
};

// Device arrays of a fused launch: descriptors, tile list, work counter.
struct Aux {
  uint64_t off = 0, bytes = 0;
  const SolveDesc* descs = nullptr;
  const int2* tiles = nullptr;
  uint32_t* counter = nullptr;
  int n_tiles = 0, maxT = 1, maxG = 1, maxTiles = 1;
};

struct Staged {
  std::vector<std::unique_ptr<Solve>> solves;
  Aux aux;
};

struct Inflight {
  Staged st;
  hipEvent_t done = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  int stream_idx = 0;
};

// Served work ring (the persistent kernel k_served and its items; see
// ring.hpp).  One pinned block holds the tails, the lost flag, the items, the
// slots' completion words and per slot an area with the solve's upload mirror
// and its result, weights and costs as the kernel writes them; one device
// block holds the ticket and prep heads, the device copies of the tails and
// per-slot counters.
struct RingSolve {
  std::unique_ptr<Solve> s;
  uint32_t slot = 0, seq = 0, items = 0;
};

struct ServedRing {
  bool on = false;
  char* pin = nullptr;
  size_t pin_bytes = 0;
  intptr_t dev_delta = 0;        // device address of pinned memory minus host address
  char* dev = nullptr;
  uint64_t* tail = nullptr;
  uint64_t* ptail = nullptr;
  uint32_t* lost = nullptr;
  uint32_t* done = nullptr;
  RingItem* items = nullptr;     // tile queue
  RingItem* pitems = nullptr;    // prep queue
  uint32_t cap = 0, pcap = 0, nslots = 0, grid = 1;
  int max_tiles = 1;
  size_t area_off = 0, slot_bytes = 0, o_res = 0, o_wn = 0, o_J = 0;   // upload mirror at 0
  uint64_t published = 0, in_use = 0, published_p = 0;
  uint32_t next_seq = 1;
  std::vector<uint32_t> free_slots;
  std::vector<RingSolve> live;
  hipEvent_t ev = nullptr;
  bool running = false;
  bool closing = false;          // exit items of the running launch published
  uint64_t quiet_since = 0;      // no live solve since then (ns)
  RingArgs args{};
  char* area(uint32_t slot) const { return pin + area_off + (size_t)slot * slot_bytes; }
  template <class T> T* on_device(void* host) const { return (T*)((intptr_t)host + dev_delta); }
};
// A launch ends after this long without live solves; polls of a waiting
// workgroup (about 1 us each) before it gives up; the device's reads of the
// host tails are at least this many 10 ns ticks apart.
constexpr uint64_t kRingQuietNs = 2000000;
constexpr uint32_t kRingWaitPolls = 1u << 23;
constexpr uint32_t kRingRefreshTicks = 100;

}  // namespace

struct mppi_engine {
  mppi_config cfg{};
  int H = 0, L = 0;
  int dev = 0;
  bool fused = false;
  std::vector<hipStream_t> streams;   // [0]: blocking path and batches; 1..: served batches
  bool own_stream0 = false;
  char* pool = nullptr;
  uint64_t pool_bytes = 0;
  bool own_pool = false;
  Arena arena;
  void* wmem = nullptr;
  DeviceWeights dw{};
  double* instU = nullptr;      // max_instances x T_max x 4
  uint32_t* instTick = nullptr;
  float* instCf = nullptr;      // MLP: max_instances x G_max x H folded latents (object permanence)
  IdTable inst_map;             // instance id -> slot (sized at create)
  std::vector<InstInfo> inst;
  std::vector<double> hover;    // T_max x 4
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  char* pin[4] = {nullptr, nullptr, nullptr, nullptr};   // pinned staging per stream
  size_t pin_cap[4] = {0, 0, 0, 0};
  // mppi_step_noalloc: the device's library-owned scratch array (address
  // looked up at create) and pinned host staging sized at create for the
  // largest solve the config accepts
  void* scratch = nullptr;
  char* pin_na = nullptr;
  size_t pin_na_bytes = 0;
  mppi_stats stats{};
  // H = 512 decoder: region size per (precision, H, G, T) of a launch, tuned
  // on the first launch of that shape unless the config fixes it
  std::unordered_map<uint64_t, int> wide_tuned;
  std::atomic<int> sticky{0};
  std::mutex mu;                // guards everything above and below
  // served path
  std::thread sched;
  std::condition_variable cv;
  bool stop = false;
  std::unique_ptr<Admission> adm;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, OwnedRequest> pending;
  std::vector<Inflight> inflight;
  std::unordered_map<uint64_t, std::unique_ptr<Solve>> done;
  std::unordered_map<uint64_t, uint64_t> ticket_submit_ns;
  ServedRing ring;              // served path through the work ring (fused, H <= 256)
};

struct mppi_batch {
  Staged st;
  hipEvent_t t0 = nullptr, t1 = nullptr, s0 = nullptr, s1 = nullptr;
  bool launched = false;
  uint64_t reserved = 0;   // budget held until mppi_batch_destroy
};

namespace {

int dev_fail(mppi_engine* e, hipError_t err) {
  if (err != hipSuccess) {
    e->sticky.store(MPPI_EDEVICE);
    return MPPI_EDEVICE;
  }
  return MPPI_OK;
}

#define HIPCHK(e, x)                                    \
  do {                                                  \
    hipError_t err_ = (x);                              \
    if (err_ != hipSuccess) return dev_fail((e), err_); \
  } while (0)

// ---------------------------------------------------------------- validation
int cholesky4(const double S[16], double Lo[16]) {
  double scale = 0.0;
  for (int i = 0; i < 16; ++i) {
    if (!isfin(S[i])) return MPPI_EINVAL;
    scale = std::max(scale, fabs(S[i]));
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < i; ++j)
      if (fabs(S[i * 4 + j] - S[j * 4 + i]) > 1e-12 * std::max(scale, 1.0)) return MPPI_EINVAL;
  for (int i = 0; i < 16; ++i) Lo[i] = 0.0;
  bool diag = true;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      if (i != j && S[i * 4 + j] != 0.0) diag = false;
  if (diag) {
    for (int i = 0; i < 4; ++i) {
      if (S[i * 5] < 0.0) return MPPI_EINVAL;
      Lo[i * 5] = sqrt(S[i * 5]);
    }
    return MPPI_OK;
  }
  const double tol = 1e-12 * std::max(scale, 1e-300);
  for (int j = 0; j < 4; ++j) {
    double d = S[j * 4 + j];
    for (int k = 0; k < j; ++k) d -= Lo[j * 4 + k] * Lo[j * 4 + k];
    if (d < -tol) return MPPI_EINVAL;
    const double ljj = d > tol ? sqrt(d) : 0.0;
    Lo[j * 4 + j] = ljj;
    for (int i = j + 1; i < 4; ++i) {
      double s = S[i * 4 + j];
      for (int k = 0; k < j; ++k) s -= Lo[i * 4 + k] * Lo[j * 4 + k];
      if (ljj == 0.0) {
        if (fabs(s) > 1e-9 * std::max(scale, 1e-300)) return MPPI_EINVAL;
        Lo[i * 4 + j] = 0.0;
      } else {
        Lo[i * 4 + j] = s / ljj;
      }
    }
  }
  return MPPI_OK;
}

int validate(const mppi_engine* e, const mppi_request* r, double Lo[16]) {
  const mppi_config& c = e->cfg;
  if (!r) return MPPI_EINVAL;
  if (r->K < 1 || r->K > c.K_max || r->T < 1 || r->T > c.T_max || r->G < 1 || r->G > c.G_max)
    return MPPI_EINVAL;
  if (!isfin(r->dt) || r->dt <= 0.0) return MPPI_EINVAL;
  if (!isfin(r->lambda) || r->lambda <= 0.0) return MPPI_EINVAL;
  for (int i = 0; i < 13; ++i)
    if (!isfin(r->x0[i])) return MPPI_EINVAL;
  if (c.dynamics == MPPI_DYN_ROTOR_RATES)
    for (int i = 0; i < 4; ++i)
      if (!(r->thrust0[i] >= 0.0 && r->thrust0[i] <= c.thrust_max)) return MPPI_EINVAL;
  const double qn = sqrt(r->x0[3] * r->x0[3] + r->x0[4] * r->x0[4] + r->x0[5] * r->x0[5] +
                         r->x0[6] * r->x0[6]);
  if (fabs(qn - 1.0) > 1e-6) return MPPI_EINVAL;
  const double wts[5] = {r->Q_gate, r->Q_vis, r->Q_sdf, r->d_safe, r->R_u};
  for (double v : wts)
    if (std::isnan(v)) return MPPI_EINVAL;
  if (!isfin(r->d_safe)) return MPPI_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (!isfin(r->wp[i])) return MPPI_EINVAL;
  if (r->U_nom)
    for (int i = 0; i < 4 * r->T; ++i)
      if (!isfin(r->U_nom[i])) return MPPI_EINVAL;
  if (!r->gates) return MPPI_EINVAL;
  for (int g = 0; g < r->G; ++g) {
    // an unobserved gate (MLP, z == NULL) takes the instance's cached frame
    // and latent; whether there is one is checked once the instance's slot
    // is known (stage)
    if (!r->gates[g].z) {
      if (c.sdf_kind != MPPI_SDF_MLP) return MPPI_EINVAL;
      continue;
    }
    for (int i = 0; i < 9; ++i)
      if (!isfin(r->gates[g].R[i])) return MPPI_EINVAL;
    for (int i = 0; i < 3; ++i)
      if (!isfin(r->gates[g].t[i])) return MPPI_EINVAL;
    if (c.sdf_kind == MPPI_SDF_MLP)
      for (int i = 0; i < c.latent_dim; ++i)
        if (!std::isfinite(r->gates[g].z[i])) return MPPI_EINVAL;
  }
  return cholesky4(r->Sigma, Lo);
}

// ---------------------------------------------------------------- instances
int acquire_slot(mppi_engine* e, uint64_t id, int* slot) {
  const int found = e->inst_map.find(id);
  if (found >= 0) {
    *slot = found;
    return MPPI_OK;
  }
  if ((int)e->inst.size() >= e->cfg.max_instances) return MPPI_EAGAIN;
  const int s = (int)e->inst.size();
  // a new instance starts from hover with tick 0: every slot of the table is
  // filled with hover and tick 0 at create, so no copy is needed here
  InstInfo info;
  info.id = id;
  info.U_len = e->cfg.T_max;
  info.busy = false;
  e->inst.push_back(info);        // capacity reserved at create: no reallocation
  e->inst_map.insert(id, s);
  *slot = s;
  return MPPI_OK;
}

// Every unobserved gate of r (z == NULL) has a cached observation in its
// instance (object permanence).
bool gates_cached_ok(const mppi_engine* e, const mppi_request* r) {
  uint32_t need = 0;
  for (int g = 0; g < r->G; ++g)
    if (!r->gates[g].z) need |= 1u << g;
  if (!need) return true;
  const int slot = e->inst_map.find(r->instance_id);
  return slot >= 0 && (e->inst[slot].seen & need) == need;
}

int tile_rollouts(const mppi_engine* e, int G) {
  return fused_tile_rollouts(e->cfg.precision, e->H, G);
}

// exports: a blocking solve that returns its intermediates (plain path:
// samples, positions and field values; fused path: field values).
SolveLayout layout_for(const mppi_engine* e, int K, int T, int G, bool exports = false) {
  const int R = e->fused ? tile_rollouts(e, G) : 1;
  const int nt = e->fused ? (K + R - 1) / R : 0;
  return solve_layout(K, T, G, e->H, e->fused, nt, e->fused && exports);
}

// Device bytes one solve takes from the budget: its block, plus on the fused
// path its share of a batch's launch block (descriptor, tile list entries and
// work counter), so that the launch block of any batch fits in the budget its
// solves were admitted with.
uint64_t admission_footprint(const mppi_engine* e, int K, int T, int G, bool exports = false) {
  uint64_t fp = layout_for(e, K, T, G, exports).total;
  if (e->fused) {
    const int R = tile_rollouts(e, G);
    fp += align_up(sizeof(SolveDesc)) + align_up(sizeof(int2) * (uint64_t)((K + R - 1) / R)) + kAlign;
  }
  return fp;
}

// Fill the upload part (descriptor + request data) of a solve whose device
// block starts at `base`.  Lo is the Cholesky factor from validate().
void pack_solve(mppi_engine* e, const mppi_request* r, Solve* s, const double Lo[16], char* base,
                char* host) {
  const mppi_config& c = e->cfg;
  const int K = r->K, T = r->T, G = r->G, H = e->H;
  const SolveLayout& lay = s->lay;
  memset(host, 0, lay.upload_bytes);
  SolveDesc& d = s->desc;
  d = SolveDesc{};
  d.K = K;
  d.T = T;
  d.G = G;
  d.flags = (int32_t)r->flags;
  d.H = H;
  d.n_hidden = e->L;
  d.sdf_kind = c.sdf_kind;
  d.instance_id = r->instance_id;
  d.seed = c.seed;
  d.tick_fixed = r->tick;
  d.q_off = (r->flags & MPPI_REQ_SDF_AT_P0) ? 0u : 1u;
  d.dt = (float)r->dt;
  d.inv_mass = (float)(1.0 / c.mass);
  d.gravity = (float)c.gravity;
  for (int i = 0; i < 4; ++i) d.q0[i] = (float)r->x0[3 + i];
  for (int i = 0; i < 16; ++i) d.L[i] = (float)Lo[i];
  for (int i = 0; i < 4; ++i) {
    d.u_lo[i] = (float)c.u_lo[i];
    d.u_hi[i] = (float)c.u_hi[i];
  }
  d.Q_gate = (float)r->Q_gate;
  d.Q_vis = (float)r->Q_vis;
  d.Q_sdf = (float)r->Q_sdf;
  d.d_safe = (float)r->d_safe;
  d.R_u = (float)r->R_u;
  d.sdf_c = (float)c.sdf_c;
  d.sdf_tan_alpha = (float)c.sdf_tan_alpha;
  d.lambda = r->lambda;
  d.inv_lambda = 1.0 / r->lambda;
  const double* p0 = r->x0;
  const double* v0 = r->x0 + 7;
  const double tau = T * r->dt;
  double ev[3], vt[3];
  for (int i = 0; i < 3; ++i) {
    ev[i] = p0[i] - r->wp[i];
    vt[i] = v0[i] * tau;
    d.fprog[i] = (float)(vt[i] + ev[i]);
  }
  const double qg = r->Q_gate;
  const double c0 = vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2] +
                    2.0 * (vt[0] * ev[0] + vt[1] * ev[1] + vt[2] * ev[2]);
  d.C0 = (qg == 0.0 || c0 == 0.0) ? 0.0 : qg * c0;
  s->C0 = d.C0;
  d.hover[0] = c.dynamics == MPPI_DYN_ROTOR_RATES ? 0.0 : c.mass * c.gravity;
  d.dyn = c.dynamics;
  if (c.dynamics == MPPI_DYN_ROTOR_RATES) {
    d.rot_a = (float)(c.arm_length / std::sqrt(2.0));
    d.rot_kappa = (float)c.yaw_coeff;
    d.thrust_max = (float)c.thrust_max;
    d.rate_max = (float)c.rate_max;
    for (int i = 0; i < 3; ++i) {
      d.Jd[i] = (float)c.inertia[i];
      d.Jinv[i] = (float)(1.0 / c.inertia[i]);
      d.w0[i] = (float)r->x0[10 + i];
    }
    for (int i = 0; i < 4; ++i) d.thrust0[i] = (float)r->thrust0[i];
  }
  if (r->U_nom) {
    memcpy(host + lay.U, r->U_nom, sizeof(double) * 4 * T);
    d.U_src = (const double*)(base + lay.U);
    d.U_len = T;
  } else {
    d.U_src = e->instU + (size_t)s->slot * c.T_max * 4;
    d.U_len = e->inst[s->slot].U_len;
  }
  d.U_resident = e->instU + (size_t)s->slot * c.T_max * 4;
  d.tick_slot = e->instTick + s->slot;
  float* Rt = (float*)(host + lay.Rt);
  float* bs = (float*)(host + lay.base);
  float* zz = (float*)(host + lay.z);
  InstInfo& ii = e->inst[s->slot];
  d.cf_cache = e->instCf ? e->instCf + (size_t)s->slot * c.G_max * H : nullptr;
  d.fold_cached = 0;
  for (int g = 0; g < G; ++g) {
    const bool observed = r->gates[g].z != nullptr;
    if (observed) {
      // this request's observation becomes the instance's cached gate g
      // (its fold is stored by the fold kernel when the solve runs)
      memcpy(ii.R[g], r->gates[g].R, sizeof(ii.R[g]));
      memcpy(ii.t[g], r->gates[g].t, sizeof(ii.t[g]));
      ii.seen |= 1u << g;
    } else {
      d.fold_cached |= 1u << g;
    }
    const double* R = observed ? r->gates[g].R : ii.R[g];
    const double* tg = observed ? r->gates[g].t : ii.t[g];
    double rt[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) rt[i * 3 + j] = R[j * 3 + i];
    for (int i = 0; i < 9; ++i) Rt[g * 9 + i] = (float)rt[i];
    double o[3], rv[3];
    for (int i = 0; i < 3; ++i) {
      o[i] = 0.0;
      rv[i] = 0.0;
      for (int j = 0; j < 3; ++j) {
        o[i] += rt[i * 3 + j] * (p0[j] - tg[j]);
        rv[i] += rt[i * 3 + j] * v0[j];
      }
    }
    for (int t = 0; t <= T; ++t)
      for (int i = 0; i < 3; ++i)
        bs[((size_t)g * (T + 1) + t) * 3 + i] = (float)(o[i] + (t * r->dt) * rv[i]);
    if (c.sdf_kind == MPPI_SDF_MLP && observed) memcpy(zz + (size_t)g * kLatent, r->gates[g].z, sizeof(float) * kLatent);
  }
  float* los = (float*)(host + lay.los);
  for (int t = 0; t < T; ++t) {
    los[2 * t] = (float)(r->wp[0] - p0[0] - v0[0] * t * r->dt);
    los[2 * t + 1] = (float)(r->wp[1] - p0[1] - v0[1] * t * r->dt);
  }
  d.Rt = (const float*)(base + lay.Rt);
  d.base = (const float*)(base + lay.base);
  d.z = (const float*)(base + lay.z);
  d.cfold = (float*)(base + lay.cfold);
  d.los = (const float*)(base + lay.los);
  d.result = (double*)(base + lay.result);
  d.J = (float*)(base + lay.J);
  d.wn = s->want_w ? (double*)(base + lay.wn) : nullptr;
  if (!e->fused) {
    d.samples = (float*)(base + lay.samples);
    d.pos = (float*)(base + lay.pos);
    d.sdf = (float*)(base + lay.sdf);
    d.Jpart = (float*)(base + lay.Jpart);
    d.wt = (double*)(base + lay.wt);
  } else {
    const int R = tile_rollouts(e, G);
    d.sdf = s->exports ? (float*)(base + lay.sdf) : nullptr;
    d.partials = (double*)(base + lay.partials);
    d.tile_rollouts = R;
    d.n_tiles = (K + R - 1) / R;
  }
  memcpy(host + lay.desc, &d, sizeof(SolveDesc));
  s->dt = r->dt;
  for (int i = 0; i < 3; ++i) s->v0[i] = v0[i];
}

void release_staged(mppi_engine* e, Staged& st, bool free_instances) {
  for (auto& s : st.solves) {
    if (!s) continue;
    if (s->bytes) e->arena.release(s->off, s->bytes);
    s->bytes = 0;
    if (free_instances && s->slot >= 0) e->inst[s->slot].busy = false;
  }
  if (st.aux.bytes) e->arena.release(st.aux.off, st.aux.bytes);
  st.aux.bytes = 0;
}

// Pinned staging buffer of serving stream si with at least `bytes` capacity.
// A stream's buffer is only rewritten once that stream's previous copies
// have completed (one batch in flight per stream; blocking calls synchronise).
char* pinned_for(mppi_engine* e, int si, size_t bytes) {
  if (e->pin_cap[si] < bytes) {
    if (hipStreamSynchronize(e->streams[si]) != hipSuccess) return nullptr;
    if (e->pin[si]) hipHostFree(e->pin[si]);
    e->pin[si] = nullptr;
    e->pin_cap[si] = 0;
    const size_t cap = std::max<size_t>(bytes + bytes / 2, 1 << 20);
    if (hipHostMalloc((void**)&e->pin[si], cap, hipHostMallocDefault) != hipSuccess) return nullptr;
    e->pin_cap[si] = cap;
  }
  return e->pin[si];
}

// Validate, bind instances, allocate, pack and upload a set of requests.
// The uploads are asynchronous copies on stream si from its pinned staging
// buffer, so kernels enqueued after them on si see the data.  Every instance
// is held busy until the staged set is released.  On failure nothing stays
// allocated or held.
int stage(mppi_engine* e, const std::vector<const mppi_request*>& reqs, bool want_w, bool want_J,
          bool exports, int si, Staged& out) {
  std::unordered_set<uint64_t> ids;
  for (auto* r : reqs)
    if (!ids.insert(r->instance_id).second) return MPPI_EINVAL;   // one solve per instance at a time
  auto fail = [&](int rc) {
    release_staged(e, out, true);
    out.solves.clear();
    return rc;
  };
  std::vector<std::array<double, 16>> Lo(reqs.size());
  size_t up_total = 0;
  for (size_t i = 0; i < reqs.size(); ++i) {
    const mppi_request* r = reqs[i];
    int rc = validate(e, r, Lo[i].data());
    auto s = std::make_unique<Solve>();
    s->K = r->K;
    s->T = r->T;
    s->G = r->G;
    s->flags = r->flags;
    s->want_w = want_w;
    s->want_J = want_J;
    s->exports = exports;
    if (rc == MPPI_OK) rc = acquire_slot(e, r->instance_id, &s->slot);
    if (rc == MPPI_OK && e->inst[s->slot].busy) rc = MPPI_EAGAIN;
    if (rc == MPPI_OK && !gates_cached_ok(e, r)) rc = MPPI_EINVAL;   // a gate never observed
    if (rc == MPPI_OK) {
      s->lay = layout_for(e, r->K, r->T, r->G, exports);
      if (!e->arena.alloc(s->lay.total, &s->off)) rc = MPPI_ENOMEM;
      else s->bytes = s->lay.total;
    }
    if (rc != MPPI_OK) return fail(rc);
    e->inst[s->slot].busy = true;
    up_total += align_up(s->lay.upload_bytes);
    out.solves.push_back(std::move(s));
  }
  // fused launches also upload the descriptor array and the tile list
  std::vector<int2> tiles;
  uint64_t o_tiles = 0, o_cnt = 0;
  Aux& a = out.aux;
  if (e->fused) {
    for (size_t i = 0; i < out.solves.size(); ++i) {
      const Solve* s = out.solves[i].get();
      const int R = tile_rollouts(e, s->G);
      const int nt = (s->K + R - 1) / R;
      for (int t = 0; t < nt; ++t) tiles.push_back(int2{(int)i, t * R});
      a.maxT = std::max(a.maxT, s->T);
      a.maxG = std::max(a.maxG, s->G);
      a.maxTiles = std::max(a.maxTiles, nt);
    }
    // longest tiles first (work per tile grows with T G); ties keep solve order
    std::stable_sort(tiles.begin(), tiles.end(), [&](const int2& x, const int2& y) {
      const Solve* sx = out.solves[x.x].get();
      const Solve* sy = out.solves[y.x].get();
      return sx->T * sx->G > sy->T * sy->G;
    });
    const size_t nS = out.solves.size();
    o_tiles = align_up(sizeof(SolveDesc) * nS);
    o_cnt = o_tiles + align_up(sizeof(int2) * tiles.size());
    const uint64_t bytes = o_cnt + kAlign;
    if (!e->arena.alloc(bytes, &a.off)) return fail(MPPI_ENOMEM);
    a.bytes = bytes;
    up_total += bytes;
  }
  char* pin = pinned_for(e, si, up_total);
  if (!pin) return fail(dev_fail(e, hipErrorOutOfMemory));
  hipStream_t st = e->streams[si];
  size_t po = 0;
  for (size_t i = 0; i < reqs.size(); ++i) {
    Solve* s = out.solves[i].get();
    char* base = e->pool + s->off;
    pack_solve(e, reqs[i], s, Lo[i].data(), base, pin + po);
    const hipError_t err = hipMemcpyAsync(base, pin + po, s->lay.upload_bytes, hipMemcpyHostToDevice, st);
    if (err != hipSuccess) return fail(dev_fail(e, err));
    po += align_up(s->lay.upload_bytes);
  }
  if (e->fused) {
    char* ah = pin + po;
    memset(ah, 0, a.bytes);
    for (size_t i = 0; i < out.solves.size(); ++i)
      memcpy(ah + i * sizeof(SolveDesc), &out.solves[i]->desc, sizeof(SolveDesc));
    memcpy(ah + o_tiles, tiles.data(), sizeof(int2) * tiles.size());
    char* ab = e->pool + a.off;
    const hipError_t err = hipMemcpyAsync(ab, ah, a.bytes, hipMemcpyHostToDevice, st);
    if (err != hipSuccess) return fail(dev_fail(e, err));
    a.descs = (const SolveDesc*)ab;
    a.tiles = (const int2*)(ab + o_tiles);
    a.counter = (uint32_t*)(ab + o_cnt);
    a.n_tiles = (int)tiles.size();
  }
  return MPPI_OK;
}

// Region size of the H = 512 decoder for a launch of max shape (maxG, maxT):
// the config's, else the tuned one for (precision, H, maxG, maxT), tuned now
// (synchronously, on the batch's own inputs) when allowed, else the default.
int wide_region_for(mppi_engine* e, const FusedBatch& fb, int n_solves, int maxT, int maxG, int maxTiles,
                    hipStream_t st, bool may_tune, int* out) {
  *out = 4;
  if (e->H != 512) return MPPI_OK;
  if (e->cfg.wide_region != 0) {
    *out = e->cfg.wide_region;
  } else {
    const uint64_t key = ((uint64_t)(uint32_t)e->cfg.precision << 32) | ((uint64_t)e->H << 16) |
                         ((uint64_t)maxG << 8) | (uint64_t)maxT;
    auto it = e->wide_tuned.find(key);
    if (it != e->wide_tuned.end()) {
      *out = it->second;
    } else if (may_tune) {
      int best = 4;
      HIPCHK(e, tune_wide_region(fb, n_solves, e->dw, maxT, maxG, maxTiles, st, &best));
      e->wide_tuned[key] = best;
      e->stats.tune_runs++;
      *out = best;
    }
  }
  e->stats.wide_region = (uint64_t)*out;
  return MPPI_OK;
}

// Enqueue every kernel of a staged set on stream st.  t0/t1 (optional) bracket
// the dominant kernel(s): the SDF kernels of the plain path, the fused kernel.
int launch_staged(mppi_engine* e, Staged& sg, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (!e->fused) {
    for (size_t i = 0; i < sg.solves.size(); ++i) {
      Solve* s = sg.solves[i].get();
      PlainShape shp{s->K, s->T, s->G, e->cfg.sdf_kind};
      const bool first = i == 0, last = i + 1 == sg.solves.size();
      HIPCHK(e, launch_plain((const SolveDesc*)(e->pool + s->off + s->lay.desc), shp, e->dw, st,
                             first ? t0 : nullptr, last ? t1 : nullptr));
    }
    return MPPI_OK;
  }
  Aux& a = sg.aux;
  FusedBatch fb{a.descs, a.tiles, a.n_tiles, a.counter};
  int rg = 4;
  const int rc = wide_region_for(e, fb, (int)sg.solves.size(), a.maxT, a.maxG, a.maxTiles, st, true, &rg);
  if (rc != MPPI_OK) return rc;
  HIPCHK(e, launch_fused(fb, (int)sg.solves.size(), e->dw, a.maxT, a.maxG, a.maxTiles, st, t0, t1, rg));
  return MPPI_OK;
}

// Enqueue the D2H copies of a solve's outputs on stream st.
int enqueue_fetch(mppi_engine* e, Solve* s, hipStream_t st) {
  const int K = s->K, T = s->T;
  char* base = e->pool + s->off;
  s->res.resize(4 * T + RES_SCALARS);
  HIPCHK(e, hipMemcpyAsync(s->res.data(), base + s->lay.result, sizeof(double) * s->res.size(),
                           hipMemcpyDeviceToHost, st));
  if (s->want_w) {
    s->wn.resize(K);
    HIPCHK(e, hipMemcpyAsync(s->wn.data(), base + s->lay.wn, sizeof(double) * K, hipMemcpyDeviceToHost, st));
  }
  if (s->want_J) {
    s->J.resize(K);
    HIPCHK(e, hipMemcpyAsync(s->J.data(), base + s->lay.J, sizeof(float) * K, hipMemcpyDeviceToHost, st));
  }
  if (s->exports) {
    if (!e->fused) {
      s->samples.resize((size_t)4 * T * K);
      s->pos.resize((size_t)3 * (T + 1) * K);
      HIPCHK(e, hipMemcpyAsync(s->samples.data(), base + s->lay.samples, 4 * s->samples.size(),
                               hipMemcpyDeviceToHost, st));
      HIPCHK(e, hipMemcpyAsync(s->pos.data(), base + s->lay.pos, 4 * s->pos.size(), hipMemcpyDeviceToHost, st));
    }
    s->sdf.resize((size_t)T * K);
    HIPCHK(e, hipMemcpyAsync(s->sdf.data(), base + s->lay.sdf, 4 * s->sdf.size(), hipMemcpyDeviceToHost, st));
  }
  return MPPI_OK;
}

void fill_result(const Solve* s, mppi_result* out) {
  const int T = s->T, K = s->K;
  const double* r = s->res.data();
  const double* sc = r + 4 * T;
  out->status = (int32_t)sc[RES_STATUS];
  out->tick_used = (uint32_t)sc[RES_TICK];
  if (out->U_star) memcpy(out->U_star, r, sizeof(double) * 4 * T);
  for (int c = 0; c < 4; ++c) out->u0[c] = sc[RES_U0 + c];
  out->J_min = sc[RES_JMIN];
  out->log_eta = sc[RES_LOGETA];
  out->ess = sc[RES_ESS];
  if (out->weights && s->want_w && (int)s->wn.size() == K) memcpy(out->weights, s->wn.data(), sizeof(double) * K);
  if (out->costs && s->want_J && (int)s->J.size() == K)
    for (int k = 0; k < K; ++k) out->costs[k] = (double)s->J[k] + s->C0;
  if (s->exports) {
    const size_t TK = (size_t)T * K, T1K = (size_t)(T + 1) * K;
    if (out->samples && !s->samples.empty())
      for (int k = 0; k < K; ++k)
        for (int t = 0; t < T; ++t)
          for (int c = 0; c < 4; ++c)
            out->samples[((size_t)k * T + t) * 4 + c] = s->samples[c * TK + (size_t)t * K + k];
    if (out->positions && !s->pos.empty())
      for (int k = 0; k < K; ++k)
        for (int t = 0; t <= T; ++t)
          for (int c = 0; c < 3; ++c)
            out->positions[((size_t)k * (T + 1) + t) * 3 + c] =
                (float)((double)s->pos[c * T1K + (size_t)t * K + k] + s->v0[c] * (t * s->dt));
    if (out->sdf && !s->sdf.empty())
      for (int k = 0; k < K; ++k)
        for (int t = 0; t < T; ++t) out->sdf[(size_t)k * T + t] = s->sdf[(size_t)t * K + k];
  }
  out->t_submit_ns = s->t_submit;
  out->t_admit_ns = s->t_admit;
  out->t_done_ns = s->t_done;
}

// After a solve's results are on the host: the resident sequence's length.
void note_result(mppi_engine* e, const Solve* s) {
  if (s->res.empty() || s->slot < 0) return;
  const int st = (int)s->res[4 * s->T + RES_STATUS];
  if (st == MPPI_OK && !(s->flags & MPPI_REQ_NO_SHIFT)) e->inst[s->slot].U_len = s->T;
}

void add_time(mppi_engine* e, hipEvent_t a, hipEvent_t b, bool sdf) {
  float ms = 0.0f;
  if (a && b && hipEventElapsedTime(&ms, a, b) == hipSuccess) {
    if (sdf) {
      e->stats.sdf_ms += ms;
      e->stats.sdf_launches++;
    } else {
      e->stats.solve_ms += ms;
      e->stats.solve_launches++;
    }
  }
}

// ---------------------------------------------------------------- weights
int upload_weights(mppi_engine* e, const mppi_sdf_weights* w) {
  const int H = e->H, L = e->L, D = e->cfg.latent_dim;
  const int nh = std::max(L - 1, 1);  // hidden H x H layers
  const int NF = 3 + 6 * e->cfg.pe_freqs;   // encoded-point columns of layer 0
  const int KQ = e->cfg.pe_freqs > 0 ? (NF + 3) / 4 : 0;
  std::vector<float> w1pe((size_t)H * 4 * KQ, 0.0f);
  const bool mlp = e->cfg.sdf_kind == MPPI_SDF_MLP;
  std::vector<float> w1p((size_t)H * 4, 0.0f), hbias((size_t)nh * H, 0.0f), wout(H, 0.0f);
  std::vector<double> w0lat((size_t)H * D, 0.0), b0(H, 0.0);
  std::vector<float> hf32;
  std::vector<uint8_t> hlp, pe16;
  float pe16_scale = 1.0f;
  std::vector<float> wsc(nh, 1.0f), asc(nh, 1.0f), ainv(nh, 1.0f);
  float bout = 0.0f;
  if (mlp) {
    for (int m = 0; m < H; ++m) {
      for (int i = 0; i < 3; ++i) w1p[m * 4 + i] = w->W[0][(size_t)m * (NF + D) + i];
      for (int j = 0; j < D; ++j) w0lat[(size_t)j * H + m] = w->W[0][(size_t)m * (NF + D) + NF + j];
      b0[m] = w->b[0][m];
    }
    // encoded-point columns as 16x16x4 operand fragments [mb][ks][lane]
    for (int mb = 0; mb < H / 16 && KQ > 0; ++mb)
      for (int ks = 0; ks < KQ; ++ks)
        for (int lane = 0; lane < 64; ++lane) {
          const int m = 16 * mb + lane % 16, f = 4 * ks + lane / 16;
          if (f < NF) w1pe[((size_t)mb * KQ + ks) * 64 + lane] = w->W[0][(size_t)m * (NF + D) + f];
        }
    for (int l = 0; l < L - 1; ++l)
      for (int m = 0; m < H; ++m) hbias[(size_t)l * H + m] = w->b[l + 1][m];
    for (int m = 0; m < H; ++m) wout[m] = w->W[L][m];
    bout = w->b[L][0];
    if (e->cfg.precision == MPPI_PREC_FP32 && !e->fused) {
      // 16x16x4 FP32 operand fragments: [mb][ks][lane] = W[16 mb + lane % 16][4 ks + lane / 16]
      hf32.resize((size_t)(L - 1) * H * H);
      for (int l = 0; l < L - 1; ++l) {
        const float* W = w->W[l + 1];
        float* P = &hf32[(size_t)l * H * H];
        for (int mb = 0; mb < H / 16; ++mb)
          for (int ks = 0; ks < H / 4; ++ks)
            for (int lane = 0; lane < 64; ++lane)
              P[((size_t)mb * (H / 4) + ks) * 64 + lane] = W[(size_t)(16 * mb + lane % 16) * H + 4 * ks + lane / 16];
      }
    }
    if (e->fused) {
      int rc = pack_lowp_weights(e->cfg.precision, H, L, w, hlp, wsc, asc, ainv);
      if (rc != MPPI_OK) return rc;
      if (KQ > 0) pack_pe_weights_f16(H, NF, NF + D, w->W[0], pe16, pe16_scale);
    }
  }
  const uint64_t o_w1p = 0;
  const uint64_t o_hb = align_up(o_w1p + 4 * w1p.size());
  const uint64_t o_wo = align_up(o_hb + 4 * hbias.size());
  const uint64_t o_w0 = align_up(o_wo + 4 * wout.size());
  const uint64_t o_b0 = align_up(o_w0 + 8 * w0lat.size());
  const uint64_t o_hf = align_up(o_b0 + 8 * b0.size());
  const uint64_t o_lp = align_up(o_hf + 4 * hf32.size());
  const uint64_t o_ws = align_up(o_lp + hlp.size());
  const uint64_t o_as = align_up(o_ws + 4 * wsc.size());
  const uint64_t o_ai = align_up(o_as + 4 * asc.size());
  const uint64_t o_pe = align_up(o_ai + 4 * ainv.size());
  const uint64_t o_p16 = align_up(o_pe + 4 * w1pe.size());
  const uint64_t total = align_up(o_p16 + pe16.size());
  HIPCHK(e, hipMalloc(&e->wmem, total));
  char* b = (char*)e->wmem;
  HIPCHK(e, hipMemcpy(b + o_w1p, w1p.data(), 4 * w1p.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_hb, hbias.data(), 4 * hbias.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_wo, wout.data(), 4 * wout.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_w0, w0lat.data(), 8 * w0lat.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_b0, b0.data(), 8 * b0.size(), hipMemcpyHostToDevice));
  if (!hf32.empty()) HIPCHK(e, hipMemcpy(b + o_hf, hf32.data(), 4 * hf32.size(), hipMemcpyHostToDevice));
  if (!hlp.empty()) HIPCHK(e, hipMemcpy(b + o_lp, hlp.data(), hlp.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_ws, wsc.data(), 4 * wsc.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_as, asc.data(), 4 * asc.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_ai, ainv.data(), 4 * ainv.size(), hipMemcpyHostToDevice));
  if (!w1pe.empty()) HIPCHK(e, hipMemcpy(b + o_pe, w1pe.data(), 4 * w1pe.size(), hipMemcpyHostToDevice));
  if (!pe16.empty()) HIPCHK(e, hipMemcpy(b + o_p16, pe16.data(), pe16.size(), hipMemcpyHostToDevice));
  DeviceWeights& dw = e->dw;
  dw.H = H;
  dw.n_hidden = L;
  dw.precision = e->cfg.precision;
  dw.w1p = (const float*)(b + o_w1p);
  dw.hbias = (const float*)(b + o_hb);
  dw.wout = (const float*)(b + o_wo);
  dw.w0lat = (const double*)(b + o_w0);
  dw.b0 = (const double*)(b + o_b0);
  dw.bout = bout;
  dw.hidden_f32 = hf32.empty() ? nullptr : (const float*)(b + o_hf);
  dw.hidden_lp = hlp.empty() ? nullptr : (const void*)(b + o_lp);
  dw.w_scale = (const float*)(b + o_ws);
  dw.a_scale = (const float*)(b + o_as);
  dw.a_inv = (const float*)(b + o_ai);
  dw.pe_freqs = e->cfg.pe_freqs;
  dw.n_feat = NF;
  dw.feat_ksteps = KQ;
  dw.w1pe = w1pe.empty() ? nullptr : (const float*)(b + o_pe);
  dw.feat_k32 = KQ > 0 ? (NF + 31) / 32 : 0;
  dw.w1pe_scale = pe16_scale;
  dw.w1pe16 = pe16.empty() ? nullptr : (const void*)(b + o_p16);
  return MPPI_OK;
}

void scheduler_loop(mppi_engine* e);
int ring_setup(mppi_engine* e);
void ring_free(mppi_engine* e);
int ring_end_launch(mppi_engine* e);

}  // namespace

extern "C" {

const char* mppi_status_str(int s) {
  switch (s) {
    case MPPI_OK: return "ok";
    case MPPI_PENDING: return "pending";
    case MPPI_EINVAL: return "invalid argument";
    case MPPI_ENOMEM: return "out of device memory or over the budget";
    case MPPI_EAGAIN: return "queue full, instance busy or no free instance slot: retry";
    case MPPI_ENOTFOUND: return "unknown or retired ticket";
    case MPPI_ENUMERIC: return "every rollout cost is non-finite";
    case MPPI_EDEVICE: return "HIP device error";
    default: return "unknown status";
  }
}

int mppi_create(const mppi_config* cfg, const mppi_sdf_weights* w, mppi_engine** out) {
  if (!cfg || !out) return MPPI_EINVAL;
  const mppi_config& c = *cfg;
  if (c.precision < 0 || c.precision > 5 || c.path < 0 || c.path > 1 || c.sdf_kind < 0 || c.sdf_kind > 1)
    return MPPI_EINVAL;
  if (c.latent_dim != kLatent) return MPPI_EINVAL;
  if (c.sdf_kind == MPPI_SDF_MLP) {
    if (!(c.hidden == 64 || c.hidden == 128 || c.hidden == 256 || c.hidden == 512)) return MPPI_EINVAL;
    if (c.n_hidden < 2 || c.n_hidden > 8) return MPPI_EINVAL;
    if (!w || !w->W || !w->b) return MPPI_EINVAL;
    for (int l = 0; l <= c.n_hidden; ++l)
      if (!w->W[l] || !w->b[l]) return MPPI_EINVAL;
    if (c.precision == MPPI_PREC_FP8 && !w->act_scale) return MPPI_EINVAL;
  }
  if (c.precision == MPPI_PREC_BF16X3 && c.path != MPPI_PATH_FUSED) return MPPI_EINVAL;
  if (c.path == MPPI_PATH_PLAIN && c.precision != MPPI_PREC_FP32) return MPPI_EINVAL;
  if (c.path == MPPI_PATH_FUSED) {
    if (c.sdf_kind != MPPI_SDF_MLP || !fused_supported(c.precision, c.hidden, c.n_hidden)) return MPPI_EINVAL;
    const int max_tiles = (c.K_max + fused_tile_rollouts(c.precision, c.hidden, c.G_max) - 1) /
                          fused_tile_rollouts(c.precision, c.hidden, c.G_max);
    const int feat_ks = c.pe_freqs > 0 ? (3 + 6 * c.pe_freqs + 31) / 32 : 0;   // 32-wide K-steps of the encoded point
    if (fused_lds_bytes(c.precision, c.hidden, c.n_hidden, c.T_max, c.G_max, max_tiles, feat_ks) > kMaxLdsBytes)
      return MPPI_EINVAL;
  }
  if (c.K_max < 1 || c.K_max > kMaxK || c.T_max < 1 || c.T_max > kMaxT || c.G_max < 1 || c.G_max > kMaxG)
    return MPPI_EINVAL;
  if (c.max_instances < 1 || c.max_inflight < 1 || c.queue_depth < 1) return MPPI_EINVAL;
  if (c.wide_region != 0 && c.wide_region != 2 && c.wide_region != 4 && c.wide_region != 8) return MPPI_EINVAL;
  if (!(c.mass > 0.0) || !isfin(c.mass) || !isfin(c.gravity)) return MPPI_EINVAL;
  for (int i = 0; i < 4; ++i)
    if (!isfin(c.u_lo[i]) || !isfin(c.u_hi[i]) || c.u_lo[i] > c.u_hi[i]) return MPPI_EINVAL;
  if (!c.device_pool && c.hbm_budget_bytes == 0) return MPPI_EINVAL;
  if (c.dynamics != MPPI_DYN_CTBR && c.dynamics != MPPI_DYN_ROTOR_RATES) return MPPI_EINVAL;
  if (c.pe_freqs < 0 || c.pe_freqs > 8) return MPPI_EINVAL;
  if (c.pe_freqs > 0 && (c.sdf_kind != MPPI_SDF_MLP || (c.path == MPPI_PATH_FUSED && c.hidden > 256)))
    return MPPI_EINVAL;
  if (c.dynamics == MPPI_DYN_ROTOR_RATES) {
    for (int i = 0; i < 3; ++i)
      if (!(c.inertia[i] > 0.0) || !isfin(c.inertia[i])) return MPPI_EINVAL;
    if (!(c.arm_length > 0.0) || !isfin(c.arm_length) || !isfin(c.yaw_coeff)) return MPPI_EINVAL;
    if (!(c.thrust_max > 0.0) || !isfin(c.thrust_max) || !(c.rate_max > 0.0) || !isfin(c.rate_max))
      return MPPI_EINVAL;
  }

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || c.device < 0 || ndev <= c.device) return MPPI_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c.device) != hipSuccess) return MPPI_EDEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MPPI_EDEVICE;
  if (hipSetDevice(c.device) != hipSuccess) return MPPI_EDEVICE;

  auto e = std::make_unique<mppi_engine>();
  e->cfg = c;
  e->dev = c.device;
  e->fused = c.path == MPPI_PATH_FUSED;
  e->H = c.sdf_kind == MPPI_SDF_MLP ? c.hidden : 64;
  e->L = c.sdf_kind == MPPI_SDF_MLP ? c.n_hidden : 2;
  auto bail = [&](int rc) {
    for (size_t i = 0; i < e->streams.size(); ++i)
      if (i > 0 || e->own_stream0) hipStreamDestroy(e->streams[i]);
    for (auto& ev : e->ev)
      if (ev) hipEventDestroy(ev);
    if (e->own_pool && e->pool) hipFree(e->pool);
    if (e->wmem) hipFree(e->wmem);
    if (e->instU) hipFree(e->instU);
    if (e->instTick) hipFree(e->instTick);
    if (e->instCf) hipFree(e->instCf);
    if (e->pin_na) hipHostFree(e->pin_na);
    ring_free(e.get());
    return rc;
  };
  hipStream_t s0 = (hipStream_t)c.stream;
  if (!s0) {
    if (hipStreamCreateWithFlags(&s0, hipStreamNonBlocking) != hipSuccess) return bail(MPPI_EDEVICE);
    e->own_stream0 = true;
  }
  e->streams.push_back(s0);
  for (int i = 0; i < 3; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return bail(MPPI_EDEVICE);
    e->streams.push_back(s);
  }
  for (auto& ev : e->ev)
    if (hipEventCreate(&ev) != hipSuccess) return bail(MPPI_EDEVICE);
  int rc = upload_weights(e.get(), w);
  if (rc != MPPI_OK) return bail(rc);
  if (c.device_pool) {
    e->pool = (char*)c.device_pool;
    e->pool_bytes = c.device_pool_bytes;
  } else {
    // headroom above the admission budget for batch descriptor blocks and
    // allocator fragmentation
    e->pool_bytes = c.hbm_budget_bytes + std::max<uint64_t>(c.hbm_budget_bytes / 8, 16ull << 20);
    if (hipMalloc(&e->pool, e->pool_bytes) != hipSuccess) return bail(MPPI_ENOMEM);
    e->own_pool = true;
  }
  e->arena.reset(e->pool_bytes);
  const size_t nI = (size_t)c.max_instances;
  if (hipMalloc(&e->instU, sizeof(double) * 4 * c.T_max * nI) != hipSuccess) return bail(MPPI_ENOMEM);
  if (hipMalloc(&e->instTick, sizeof(uint32_t) * nI) != hipSuccess) return bail(MPPI_ENOMEM);
  if (hipMemset(e->instTick, 0, sizeof(uint32_t) * nI) != hipSuccess) return bail(MPPI_EDEVICE);
  if (c.sdf_kind == MPPI_SDF_MLP) {
    const size_t cf = sizeof(float) * nI * c.G_max * e->H;
    if (hipMalloc(&e->instCf, cf) != hipSuccess) return bail(MPPI_ENOMEM);
    if (hipMemset(e->instCf, 0, cf) != hipSuccess) return bail(MPPI_EDEVICE);
  }
  e->inst.reserve((size_t)c.max_instances);
  e->inst_map.reset(c.max_instances);
  // the no-allocation entry point's device scratch (this device is current)
  // and its host staging: uploads, launch block and read-back of one solve
  if (scratch_device_address(c.device, &e->scratch) != hipSuccess) return bail(MPPI_EDEVICE);
  {
    const int R = e->fused ? tile_rollouts(e.get(), c.G_max) : 1;
    const uint64_t nt = e->fused ? (uint64_t)(c.K_max + R - 1) / R : 0;
    e->pin_na_bytes = align_up(layout_for(e.get(), c.K_max, c.T_max, c.G_max).upload_bytes) +
                      align_up(sizeof(SolveDesc)) + align_up(sizeof(int2) * nt) + kAlign +
                      align_up(sizeof(double) * (4 * (uint64_t)c.T_max + RES_SCALARS)) +
                      align_up(sizeof(float) * (uint64_t)c.K_max) + align_up(sizeof(double) * (uint64_t)c.K_max);
    if (hipHostMalloc((void**)&e->pin_na, e->pin_na_bytes, hipHostMallocDefault) != hipSuccess)
      return bail(MPPI_ENOMEM);
  }
  e->hover.assign((size_t)4 * c.T_max, 0.0);
  // a new instance starts from hover: thrust m g at zero body rate, or zero
  // rotor-thrust rates (the thrusts stay where the request puts them)
  if (c.dynamics != MPPI_DYN_ROTOR_RATES)
    for (int t = 0; t < c.T_max; ++t) e->hover[4 * t] = c.mass * c.gravity;
  {
    // every instance slot starts at hover
    std::vector<double> all(e->hover.size() * nI);
    for (size_t i = 0; i < nI; ++i) memcpy(all.data() + i * e->hover.size(), e->hover.data(), sizeof(double) * e->hover.size());
    if (hipMemcpy(e->instU, all.data(), sizeof(double) * all.size(), hipMemcpyHostToDevice) != hipSuccess)
      return bail(MPPI_EDEVICE);
  }
  const uint64_t budget = c.hbm_budget_bytes ? std::min<uint64_t>(c.hbm_budget_bytes, e->pool_bytes) : e->pool_bytes;
  e->stats.budget = budget;
  e->adm = std::make_unique<Admission>(budget, c.max_inflight, c.queue_depth);
  // served requests go through the work ring where the persistent kernel
  // exists for this decoder (H <= 256) unless the config asks for batches
  if (e->fused && !(c.flags & MPPI_CFG_SERVE_BATCHES)) {
    const int tr = tile_rollouts(e.get(), c.G_max);
    const int feat_ks = c.pe_freqs > 0 ? (3 + 6 * c.pe_freqs + 31) / 32 : 0;
    const size_t lds = served_lds_bytes(c.precision, c.hidden, c.n_hidden, c.T_max, c.G_max,
                                        (c.K_max + tr - 1) / tr, feat_ks);
    if (lds > 0 && lds <= kMaxLdsBytes) {
      rc = ring_setup(e.get());
      if (rc != MPPI_OK) return bail(rc);
    }
  }
  if (hipDeviceSynchronize() != hipSuccess) return bail(MPPI_EDEVICE);
  mppi_engine* raw = e.release();
  raw->sched = std::thread(scheduler_loop, raw);
  *out = raw;
  return MPPI_OK;
}

int mppi_destroy(mppi_engine* e) {
  if (!e) return MPPI_EINVAL;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    e->stop = true;
  }
  e->cv.notify_all();
  if (e->sched.joinable()) e->sched.join();
  hipSetDevice(e->dev);
  for (auto& s : e->streams) hipStreamSynchronize(s);
  for (auto& ev : e->ev)
    if (ev) hipEventDestroy(ev);
  for (size_t i = 0; i < e->streams.size(); ++i)
    if (i > 0 || e->own_stream0) hipStreamDestroy(e->streams[i]);
  if (e->own_pool && e->pool) hipFree(e->pool);
  if (e->wmem) hipFree(e->wmem);
  if (e->instU) hipFree(e->instU);
  if (e->instTick) hipFree(e->instTick);
  if (e->instCf) hipFree(e->instCf);
  for (char* p : e->pin)
    if (p) hipHostFree(p);
  if (e->pin_na) hipHostFree(e->pin_na);
  ring_free(e);
  delete e;
  return MPPI_OK;
}

int mppi_step(mppi_engine* e, const mppi_request* r, mppi_result* out) {
  if (!e || !r || !out || !out->U_star) return MPPI_EINVAL;
  if (e->sticky.load()) return MPPI_EDEVICE;
  std::lock_guard<std::mutex> lk(e->mu);
  hipSetDevice(e->dev);
  if (ring_end_launch(e) != MPPI_OK) return MPPI_EDEVICE;
  const uint64_t t_submit = now_ns();
  Staged sg;
  const bool exports = out->samples || out->positions || out->sdf;
  // the solve's memory counts against the budget the served path admits by
  if (r->K < 1 || r->K > e->cfg.K_max || r->T < 1 || r->T > e->cfg.T_max || r->G < 1 || r->G > e->cfg.G_max)
    return MPPI_EINVAL;
  const uint64_t fp = admission_footprint(e, r->K, r->T, r->G, exports);
  const int rr = e->adm->reserve(fp);
  if (rr != 0) return rr == -2 ? MPPI_ENOMEM : MPPI_EAGAIN;
  struct Unreserve {
    Admission* a;
    uint64_t b;
    ~Unreserve() { a->unreserve(b); }
  } unreserve{e->adm.get(), fp};
  int rc = stage(e, {r}, out->weights != nullptr, out->costs != nullptr, exports, 0, sg);
  if (rc != MPPI_OK) return rc;
  hipStream_t st = e->streams[0];
  const bool timing = e->cfg.flags & MPPI_CFG_TIMING;
  if (timing) hipEventRecord(e->ev[2], st);
  rc = launch_staged(e, sg, st, timing ? e->ev[0] : nullptr, timing ? e->ev[1] : nullptr);
  if (rc == MPPI_OK && timing) hipEventRecord(e->ev[3], st);
  Solve* s = sg.solves[0].get();
  if (rc == MPPI_OK) rc = enqueue_fetch(e, s, st);
  if (rc == MPPI_OK) {
    hipError_t err = hipStreamSynchronize(st);
    if (err != hipSuccess) rc = dev_fail(e, err);
  }
  if (rc != MPPI_OK) {
    release_staged(e, sg, true);
    return rc;
  }
  s->t_submit = s->t_admit = t_submit;
  s->t_done = now_ns();
  if (timing) {
    add_time(e, e->ev[0], e->ev[1], true);
    add_time(e, e->ev[2], e->ev[3], false);
  }
  fill_result(s, out);
  note_result(e, s);
  release_staged(e, sg, true);
  e->stats.completed++;
  e->stats.bytes_peak = std::max<uint64_t>(e->stats.bytes_peak, e->arena.peak());
  return out->status;
}

int mppi_submit(mppi_engine* e, const mppi_request* r, uint64_t* ticket) {
  if (!e || !r || !ticket) return MPPI_EINVAL;
  if (e->sticky.load()) return MPPI_EDEVICE;
  double Lo[16];
  std::lock_guard<std::mutex> lk(e->mu);
  int rc = validate(e, r, Lo);
  if (rc != MPPI_OK) return rc;
  const uint64_t fp = admission_footprint(e, r->K, r->T, r->G);
  const uint64_t t = e->next_ticket;
  rc = e->adm->push(AdmissionItem{t, r->instance_id, fp, (uint64_t)r->K * r->T * r->G});
  if (rc == -2) return MPPI_ENOMEM;
  if (rc == -3) return MPPI_EAGAIN;
  e->next_ticket++;
  e->pending[t].take(*r, e->cfg.latent_dim);
  e->ticket_submit_ns[t] = now_ns();
  e->stats.submitted++;
  *ticket = t;
  e->cv.notify_all();
  return MPPI_OK;
}

int mppi_poll(mppi_engine* e, uint64_t ticket, mppi_result* out) {
  if (!e || !out) return MPPI_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  auto it = e->done.find(ticket);
  if (it == e->done.end()) {
    if (e->ticket_submit_ns.count(ticket)) return e->sticky.load() ? MPPI_EDEVICE : MPPI_PENDING;
    return MPPI_ENOTFOUND;
  }
  if (!out->U_star) return MPPI_EINVAL;
  const Solve* s = it->second.get();
  fill_result(s, out);
  const int st = out->status;
  e->done.erase(it);
  e->ticket_submit_ns.erase(ticket);
  return st;
}

int mppi_drain(mppi_engine* e) {
  if (!e) return MPPI_EINVAL;
  std::unique_lock<std::mutex> lk(e->mu);
  e->cv.wait(lk, [&] {
    return e->sticky.load() != 0 || (e->adm->queued() == 0 && e->inflight.empty() && e->ring.live.empty());
  });
  return e->sticky.load() ? MPPI_EDEVICE : MPPI_OK;
}

int mppi_get_stats(mppi_engine* e, mppi_stats* out) {
  if (!e || !out) return MPPI_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  e->stats.bytes_in_use = e->arena.in_use();
  e->stats.bytes_peak = std::max<uint64_t>(e->stats.bytes_peak, e->arena.peak());
  *out = e->stats;
  return MPPI_OK;
}

void mppi_reset_stats(mppi_engine* e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(e->mu);
  const uint64_t b = e->stats.budget;
  e->stats = mppi_stats{};
  e->stats.budget = b;
}

uint64_t mppi_solve_footprint(const mppi_engine* e, int32_t K, int32_t T, int32_t G) {
  if (!e || K < 1 || T < 1 || G < 1) return 0;
  return admission_footprint(e, K, T, G);
}

int mppi_batch_create(mppi_engine* e, const mppi_request* reqs, int32_t n, mppi_batch** out) {
  if (!e || !reqs || n < 1 || !out) return MPPI_EINVAL;
  if (e->sticky.load()) return MPPI_EDEVICE;
  std::lock_guard<std::mutex> lk(e->mu);
  hipSetDevice(e->dev);
  if (ring_end_launch(e) != MPPI_OK) return MPPI_EDEVICE;   // the uploads may run as copy kernels
  auto b = std::make_unique<mppi_batch>();
  std::vector<const mppi_request*> rs;
  uint64_t fp = 0;
  for (int i = 0; i < n; ++i) {
    rs.push_back(&reqs[i]);
    const mppi_request& r = reqs[i];
    if (r.K < 1 || r.K > e->cfg.K_max || r.T < 1 || r.T > e->cfg.T_max || r.G < 1 || r.G > e->cfg.G_max)
      return MPPI_EINVAL;
    fp += admission_footprint(e, r.K, r.T, r.G);
  }
  // the staged solves hold their memory against the served path's budget
  const int rr = e->adm->reserve(fp);
  if (rr != 0) return rr == -2 ? MPPI_ENOMEM : MPPI_EAGAIN;
  b->reserved = fp;
  int rc = stage(e, rs, true, true, false, 0, b->st);
  if (rc == MPPI_OK && hipStreamSynchronize(e->streams[0]) != hipSuccess) {
    release_staged(e, b->st, true);
    e->adm->unreserve(fp);
    return dev_fail(e, hipErrorUnknown);
  }
  if (rc != MPPI_OK) {
    e->adm->unreserve(fp);
    return rc;
  }
  for (hipEvent_t* ev : {&b->t0, &b->t1, &b->s0, &b->s1})
    if (hipEventCreate(ev) != hipSuccess) {
      release_staged(e, b->st, true);
      e->adm->unreserve(fp);
      for (hipEvent_t x : {b->t0, b->t1, b->s0, b->s1})
        if (x) hipEventDestroy(x);
      return dev_fail(e, hipErrorOutOfMemory);
    }
  *out = b.release();
  return MPPI_OK;
}

int mppi_batch_run(mppi_engine* e, mppi_batch* b) {
  if (!e || !b) return MPPI_EINVAL;
  if (e->sticky.load()) return MPPI_EDEVICE;
  std::lock_guard<std::mutex> lk(e->mu);
  hipSetDevice(e->dev);
  if (ring_end_launch(e) != MPPI_OK) return MPPI_EDEVICE;
  hipStream_t st = e->streams[0];
  const bool timing = e->cfg.flags & MPPI_CFG_TIMING;
  if (timing && b->launched) {
    // fold the previous launch's times in before its events are reused
    const hipError_t err = hipEventSynchronize(b->s1);
    if (err != hipSuccess) return dev_fail(e, err);
    add_time(e, b->t0, b->t1, true);
    add_time(e, b->s0, b->s1, false);
    b->launched = false;
  }
  if (timing) hipEventRecord(b->s0, st);
  int rc = launch_staged(e, b->st, st, timing ? b->t0 : nullptr, timing ? b->t1 : nullptr);
  if (rc != MPPI_OK) return rc;
  if (timing) {
    hipEventRecord(b->s1, st);
    b->launched = true;
  }
  return MPPI_OK;
}

int mppi_batch_wait(mppi_engine* e, mppi_batch* b) {
  if (!e || !b) return MPPI_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  hipSetDevice(e->dev);
  // a ring launch started since the batch ran would hold compute units the
  // batch may still need while this call holds the lock its exits need
  if (ring_end_launch(e) != MPPI_OK) return MPPI_EDEVICE;
  const hipError_t err = hipStreamSynchronize(e->streams[0]);
  if (err != hipSuccess) return dev_fail(e, err);
  if (b->launched) {
    add_time(e, b->t0, b->t1, true);
    add_time(e, b->s0, b->s1, false);
    b->launched = false;
  }
  return MPPI_OK;
}

int mppi_batch_results(mppi_engine* e, mppi_batch* b, mppi_result* results) {
  if (!e || !b || !results) return MPPI_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  hipSetDevice(e->dev);
  if (ring_end_launch(e) != MPPI_OK) return MPPI_EDEVICE;   // the read-backs may run as copy kernels
  hipStream_t st = e->streams[0];
  for (auto& s : b->st.solves) {
    int rc = enqueue_fetch(e, s.get(), st);
    if (rc != MPPI_OK) return rc;
  }
  const hipError_t err = hipStreamSynchronize(st);
  if (err != hipSuccess) return dev_fail(e, err);
  const uint64_t t = now_ns();
  for (size_t i = 0; i < b->st.solves.size(); ++i) {
    Solve* s = b->st.solves[i].get();
    s->t_submit = s->t_admit = s->t_done = t;
    note_result(e, s);
    fill_result(s, &results[i]);
  }
  return MPPI_OK;
}

int mppi_batch_destroy(mppi_engine* e, mppi_batch* b) {
  if (!e || !b) return MPPI_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  hipSetDevice(e->dev);
  ring_end_launch(e);   // as in mppi_batch_wait; the batch is released either way
  hipStreamSynchronize(e->streams[0]);
  release_staged(e, b->st, true);
  e->adm->unreserve(b->reserved);
  for (hipEvent_t ev : {b->t0, b->t1, b->s0, b->s1})
    if (ev) hipEventDestroy(ev);
  delete b;
  return MPPI_OK;
}

int mppi_step_noalloc(mppi_engine* e, const mppi_request* r, mppi_result* out) {
  if (!e || !r || !out || !out->U_star) return MPPI_EINVAL;
  if (out->samples || out->positions || out->sdf) return MPPI_EINVAL;
  if (e->sticky.load()) return MPPI_EDEVICE;
  std::lock_guard<std::mutex> lk(e->mu);
  // one user of this device's scratch at a time within the process
  std::lock_guard<std::mutex> dk(scratch_use_mutex(e->dev));
  hipSetDevice(e->dev);
  if (ring_end_launch(e) != MPPI_OK) return MPPI_EDEVICE;
  const uint64_t t_submit = now_ns();
  double Lo[16];
  int rc = validate(e, r, Lo);
  if (rc != MPPI_OK) return rc;
  const int K = r->K, T = r->T, G = r->G;
  // the solve's block, then on the fused path its launch block (descriptor,
  // tile list, work counter), all inside the scratch array
  Solve s;
  s.K = K;
  s.T = T;
  s.G = G;
  s.flags = r->flags;
  s.want_w = out->weights != nullptr;
  s.want_J = out->costs != nullptr;
  s.exports = false;
  s.lay = layout_for(e, K, T, G);
  const int R = e->fused ? tile_rollouts(e, G) : 1;
  const int nt = e->fused ? (K + R - 1) / R : 0;
  const uint64_t o_tiles = align_up(sizeof(SolveDesc));
  const uint64_t o_cnt = o_tiles + align_up(sizeof(int2) * (uint64_t)nt);
  const uint64_t aux_bytes = e->fused ? o_cnt + kAlign : 0;
  if (s.lay.total + aux_bytes > kScratchBytes) return MPPI_ENOMEM;
  rc = acquire_slot(e, r->instance_id, &s.slot);
  if (rc != MPPI_OK) return rc;
  if (e->inst[s.slot].busy) return MPPI_EAGAIN;
  if (!gates_cached_ok(e, r)) return MPPI_EINVAL;
  char* base = (char*)e->scratch;
  char* host = e->pin_na;
  const uint64_t up = align_up(s.lay.upload_bytes);
  char* aux_host = host + up;
  char* rb = aux_host + align_up(aux_bytes);
  pack_solve(e, r, &s, Lo, base, host);
  hipStream_t st = e->streams[0];
  HIPCHK(e, hipMemcpyAsync(base, host, s.lay.upload_bytes, hipMemcpyHostToDevice, st));
  if (e->fused) {
    memset(aux_host, 0, aux_bytes);
    memcpy(aux_host, &s.desc, sizeof(SolveDesc));
    int2* tl = (int2*)(aux_host + o_tiles);
    for (int t = 0; t < nt; ++t) tl[t] = int2{0, t * R};
    char* ab = base + s.lay.total;
    HIPCHK(e, hipMemcpyAsync(ab, aux_host, aux_bytes, hipMemcpyHostToDevice, st));
    const SolveDesc* dd = (const SolveDesc*)ab;
    FusedBatch fb{dd, (const int2*)(ab + o_tiles), nt, (uint32_t*)(ab + o_cnt)};
    int rg = 4;
    const int rc = wide_region_for(e, fb, 1, T, G, nt, st, false, &rg);
    if (rc != MPPI_OK) return rc;
    HIPCHK(e, launch_fused(fb, 1, e->dw, T, G, nt, st, nullptr, nullptr, rg));
  } else {
    PlainShape shp{K, T, G, e->cfg.sdf_kind};
    HIPCHK(e, launch_plain((const SolveDesc*)(base + s.lay.desc), shp, e->dw, st, nullptr, nullptr));
  }
  // read-back into the pinned staging: result block, costs, weights
  const size_t nres = 4 * (size_t)T + RES_SCALARS;
  double* res = (double*)rb;
  float* Jh = (float*)(rb + align_up(sizeof(double) * nres));
  double* wh = (double*)((char*)Jh + align_up(sizeof(float) * (uint64_t)K));
  HIPCHK(e, hipMemcpyAsync(res, base + s.lay.result, sizeof(double) * nres, hipMemcpyDeviceToHost, st));
  if (s.want_J) HIPCHK(e, hipMemcpyAsync(Jh, base + s.lay.J, sizeof(float) * K, hipMemcpyDeviceToHost, st));
  if (s.want_w) HIPCHK(e, hipMemcpyAsync(wh, base + s.lay.wn, sizeof(double) * K, hipMemcpyDeviceToHost, st));
  HIPCHK(e, hipStreamSynchronize(st));
  const double* sc = res + 4 * T;
  out->status = (int32_t)sc[RES_STATUS];
  out->tick_used = (uint32_t)sc[RES_TICK];
  memcpy(out->U_star, res, sizeof(double) * 4 * T);
  for (int c = 0; c < 4; ++c) out->u0[c] = sc[RES_U0 + c];
  out->J_min = sc[RES_JMIN];
  out->log_eta = sc[RES_LOGETA];
  out->ess = sc[RES_ESS];
  if (s.want_w) memcpy(out->weights, wh, sizeof(double) * K);
  if (s.want_J)
    for (int k = 0; k < K; ++k) out->costs[k] = (double)Jh[k] + s.C0;
  out->t_submit_ns = out->t_admit_ns = t_submit;
  out->t_done_ns = now_ns();
  if (out->status == MPPI_OK && !(s.flags & MPPI_REQ_NO_SHIFT)) e->inst[s.slot].U_len = T;
  e->stats.completed++;
  return out->status;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------- work ring
// Pinned and device blocks of the ring, sized for max_inflight solves of the
// largest accepted shape (every slot's items fit: tile queue slots x tiles,
// prep queue one per slot).
int ring_setup(mppi_engine* e) {
  ServedRing& R = e->ring;
  const mppi_config& c = e->cfg;
  R.nslots = (uint32_t)std::min(c.max_inflight, 1024);
  const int tr = tile_rollouts(e, c.G_max);
  R.max_tiles = (c.K_max + tr - 1) / tr;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, e->dev) != hipSuccess || ncu < 1)
    return MPPI_EDEVICE;
  R.grid = (uint32_t)ncu;
  R.cap = R.nslots * (uint32_t)R.max_tiles + R.grid;   // live solves' tiles and one launch's exits
  R.pcap = R.nslots;
  size_t o = align_up(layout_for(e, c.K_max, c.T_max, c.G_max).upload_bytes);
  R.o_res = o;
  o += align_up(sizeof(double) * (4 * (size_t)c.T_max + RES_SCALARS));
  R.o_wn = o;
  o += align_up(sizeof(double) * (size_t)c.K_max);
  R.o_J = o;
  o += align_up(sizeof(float) * (size_t)c.K_max);
  R.slot_bytes = o;
  const size_t o_items = kAlign;
  const size_t o_pitems = align_up(o_items + sizeof(RingItem) * (size_t)R.cap);
  const size_t o_done = align_up(o_pitems + sizeof(RingItem) * (size_t)R.pcap);
  R.area_off = align_up(o_done + sizeof(uint32_t) * R.nslots);
  R.pin_bytes = R.area_off + R.slot_bytes * R.nslots;
  if (hipHostMalloc((void**)&R.pin, R.pin_bytes, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
    R.pin = nullptr;
    return MPPI_ENOMEM;
  }
  memset(R.pin, 0, R.pin_bytes);
  void* dp = nullptr;
  if (hipHostGetDevicePointer(&dp, R.pin, 0) != hipSuccess) return MPPI_EDEVICE;
  R.dev_delta = (intptr_t)dp - (intptr_t)R.pin;
  R.tail = (uint64_t*)R.pin;
  R.ptail = (uint64_t*)(R.pin + 8);
  R.lost = (uint32_t*)(R.pin + 16);
  R.items = (RingItem*)(R.pin + o_items);
  R.pitems = (RingItem*)(R.pin + o_pitems);
  R.done = (uint32_t*)(R.pin + o_done);
  const size_t dbytes = 64 + sizeof(uint32_t) * 3 * (size_t)R.nslots;
  if (hipMalloc((void**)&R.dev, dbytes) != hipSuccess) {
    R.dev = nullptr;
    return MPPI_ENOMEM;
  }
  if (hipMemset(R.dev, 0, dbytes) != hipSuccess) return MPPI_EDEVICE;
  if (hipEventCreateWithFlags(&R.ev, hipEventDisableTiming) != hipSuccess) {
    R.ev = nullptr;
    return MPPI_EDEVICE;
  }
  RingArgs& a = R.args;
  a.pool = e->pool;
  a.items = R.on_device<const RingItem>(R.items);
  a.pitems = R.on_device<const RingItem>(R.pitems);
  a.tail = R.on_device<const uint64_t>(R.tail);
  a.ptail = R.on_device<const uint64_t>(R.ptail);
  a.lost = R.on_device<uint32_t>(R.lost);
  a.done = R.on_device<uint32_t>(R.done);
  a.head = (uint64_t*)R.dev;
  a.phead = (uint64_t*)(R.dev + 8);
  a.dtail = (uint64_t*)(R.dev + 16);
  a.dptail = (uint64_t*)(R.dev + 24);
  a.poll_time = (uint64_t*)(R.dev + 32);
  a.poll = (uint32_t*)(R.dev + 40);
  a.prep = (uint32_t*)(R.dev + 64);
  a.tiles = a.prep + R.nslots;
  a.fail = a.tiles + R.nslots;
  a.cap = R.cap;
  a.pcap = R.pcap;
  a.refresh_ticks = kRingRefreshTicks;
  a.wait_polls = kRingWaitPolls;
  R.free_slots.clear();
  for (uint32_t i = 0; i < R.nslots; ++i) R.free_slots.push_back(R.nslots - 1 - i);
  R.on = true;
  return MPPI_OK;
}

void ring_free(mppi_engine* e) {
  ServedRing& R = e->ring;
  if (R.ev) hipEventDestroy(R.ev);
  if (R.dev) hipFree(R.dev);
  if (R.pin) hipHostFree(R.pin);
  R.ev = nullptr;
  R.dev = nullptr;
  R.pin = nullptr;
  R.on = false;
}

// A ticket that fails before it reaches the device: its result carries rc.
void fail_ticket(mppi_engine* e, const AdmissionItem& a, int rc) {
  auto s = std::make_unique<Solve>();
  s->ticket = a.ticket;
  s->T = e->pending[a.ticket].req.T;
  s->res.assign(4 * s->T + RES_SCALARS, 0.0);
  s->res[4 * s->T + RES_STATUS] = rc;
  s->want_w = s->want_J = false;
  s->t_submit = e->ticket_submit_ns[a.ticket];
  s->t_done = now_ns();
  e->adm->complete(a.footprint);
  e->stats.failed++;
  e->done[a.ticket] = std::move(s);
  e->pending.erase(a.ticket);
}

// Validate, bind the instance, allocate the device block and pack one request
// into the pinned mirror of ring slot `slot`; its descriptor sends the result,
// the weights and a copy of the costs to the slot's pinned areas.
int ring_stage(mppi_engine* e, const mppi_request* r, uint32_t slot, std::unique_ptr<Solve>& out) {
  ServedRing& R = e->ring;
  double Lo[16];
  int rc = validate(e, r, Lo);
  auto s = std::make_unique<Solve>();
  s->K = r->K;
  s->T = r->T;
  s->G = r->G;
  s->flags = r->flags;
  s->want_w = s->want_J = true;
  s->exports = false;
  if (rc == MPPI_OK) rc = acquire_slot(e, r->instance_id, &s->slot);
  if (rc == MPPI_OK && e->inst[s->slot].busy) rc = MPPI_EAGAIN;
  if (rc == MPPI_OK && !gates_cached_ok(e, r)) rc = MPPI_EINVAL;
  if (rc == MPPI_OK) {
    s->lay = layout_for(e, r->K, r->T, r->G, false);
    if (!e->arena.alloc(s->lay.total, &s->off)) return MPPI_ENOMEM;
    s->bytes = s->lay.total;
  }
  if (rc != MPPI_OK) return rc;
  e->inst[s->slot].busy = true;
  char* area = R.area(slot);
  pack_solve(e, r, s.get(), Lo, e->pool + s->off, area);
  SolveDesc& d = s->desc;
  d.result = R.on_device<double>(area + R.o_res);
  d.wn = R.on_device<double>(area + R.o_wn);
  d.J_copy = R.on_device<float>(area + R.o_J);
  memcpy(area + s->lay.desc, &d, sizeof(SolveDesc));
  out = std::move(s);
  return MPPI_OK;
}

// Items of a staged solve: its prep item into the prep queue, one item per
// tile into the tile queue (published by the caller).
void ring_write_items(mppi_engine* e, RingSolve& rs) {
  ServedRing& R = e->ring;
  const Solve* s = rs.s.get();
  const uint64_t block = s->off;
  const uint32_t nt = (uint32_t)s->desc.n_tiles, tr = (uint32_t)s->desc.tile_rollouts;
  R.pitems[R.published_p++ % R.pcap] = RingItem{block, (uint64_t)(uintptr_t)R.on_device<char>(R.area(rs.slot)),
                                                rs.slot, -1, (uint32_t)s->lay.upload_bytes, rs.seq};
  for (uint32_t t = 0; t < nt; ++t)
    R.items[R.published++ % R.cap] = RingItem{block, 0, rs.slot, (int32_t)(t * tr), nt, rs.seq};
  rs.items = nt;
  R.in_use += rs.items;
}

// Solves whose completion word carries their sequence number: results from
// the slot's pinned areas, memory, instance and slot released.
bool ring_retire(mppi_engine* e) {
  ServedRing& R = e->ring;
  bool any = false;
  for (size_t i = 0; i < R.live.size();) {
    RingSolve& rs = R.live[i];
    const uint32_t w = __atomic_load_n(R.done + rs.slot, __ATOMIC_ACQUIRE);
    if ((w & ~kRingFailBit) != rs.seq) {
      ++i;
      continue;
    }
    Solve* s = rs.s.get();
    const char* area = R.area(rs.slot);
    const double* res = (const double*)(area + R.o_res);
    s->res.assign(res, res + 4 * s->T + RES_SCALARS);
    s->wn.assign((const double*)(area + R.o_wn), (const double*)(area + R.o_wn) + s->K);
    s->J.assign((const float*)(area + R.o_J), (const float*)(area + R.o_J) + s->K);
    if (w & kRingFailBit) {
      // a tile never saw the solve's block: the device is not trusted any
      // more, and the block stays allocated (a late copy could still land)
      s->res[4 * s->T + RES_STATUS] = MPPI_EDEVICE;
      e->sticky.store(MPPI_EDEVICE);
    } else {
      e->arena.release(s->off, s->bytes);
    }
    s->bytes = 0;
    if (s->slot >= 0) e->inst[s->slot].busy = false;
    s->t_done = now_ns();
    note_result(e, s);
    e->adm->complete(s->footprint);
    if ((int)s->res[4 * s->T + RES_STATUS] != MPPI_OK) e->stats.failed++;
    e->stats.completed++;
    R.in_use -= rs.items;
    R.free_slots.push_back(rs.slot);
    e->done[s->ticket] = std::move(rs.s);
    R.live.erase(R.live.begin() + i);
    any = true;
  }
  if (any) e->cv.notify_all();
  return any;
}

// Exit items for every workgroup of the running launch (see ring.hpp).
void ring_publish_exits(mppi_engine* e) {
  ServedRing& R = e->ring;
  for (uint32_t i = 0; i < R.grid; ++i)
    R.items[R.published++ % R.cap] = RingItem{0, 0, 0, kRingExit, 0, 0};
  __atomic_store_n(R.tail, R.published, __ATOMIC_RELEASE);
  R.closing = true;
}

// Called with the engine lock held by a path that launches kernels of its
// own (blocking solve, staged batch; the HIP runtime's copies of uploads and
// read-backs may run as kernels too): the ring kernel holds every compute
// unit while it runs, so its launch ends first.  Its exit items go behind
// everything already published, which the kernel finishes without the host;
// the scheduler retires those solves as usual.
int ring_end_launch(mppi_engine* e) {
  ServedRing& R = e->ring;
  if (!R.on || !R.running) return MPPI_OK;
  if (!R.closing) ring_publish_exits(e);
  const hipError_t err = hipEventSynchronize(R.ev);
  if (err != hipSuccess || __atomic_load_n(R.lost, __ATOMIC_ACQUIRE)) {
    e->sticky.store(MPPI_EDEVICE);
    return MPPI_EDEVICE;
  }
  R.running = false;
  R.closing = false;
  R.in_use -= R.grid;
  return MPPI_OK;
}

// Served path through the work ring.  Each pass: note whether the ring
// kernel still runs, retire completed solves, admit what fits (budget and
// ring slots) and publish it, start a launch when published work has no
// running kernel, and end the launch once no solve has been live for a
// while (or at destroy).  The kernel stays resident while work keeps coming.
void scheduler_loop_ring(mppi_engine* e) {
  hipSetDevice(e->dev);
  ServedRing& R = e->ring;
  hipStream_t st = e->streams[1];
  std::unique_lock<std::mutex> lk(e->mu);
  int idle_passes = 0;
  uint64_t stop_deadline = 0;   // destroy waits this long for running solves
  while (true) {
    const uint64_t now = now_ns();
    if (e->stop && !stop_deadline) stop_deadline = now + 30ull * 1000000000ull;
    if (stop_deadline && now > stop_deadline && !R.live.empty()) e->sticky.store(MPPI_EDEVICE);
    if (R.running) {
      const hipError_t q = hipEventQuery(R.ev);
      if (q == hipSuccess) {
        // a launch ends only through its exit items; anything else (a
        // workgroup that gave up on its ticket) leaves the ring unusable
        if (!R.closing || __atomic_load_n(R.lost, __ATOMIC_ACQUIRE)) e->sticky.store(MPPI_EDEVICE);
        R.running = false;
        R.closing = false;
        R.in_use -= R.grid;
      } else if (q != hipErrorNotReady) {
        e->sticky.store(MPPI_EDEVICE);
        R.running = false;
      }
    }
    bool progress = ring_retire(e);
    if (!R.live.empty()) R.quiet_since = now;
    if (e->stop && (R.live.empty() || e->sticky.load())) break;
    if (!e->stop && !e->sticky.load() && !R.free_slots.empty()) {
      auto adm = e->adm->admit([&](uint64_t id) {
        const int slot = e->inst_map.find(id);
        return slot >= 0 && e->inst[slot].busy;
      });
      const uint64_t tadm = now_ns();
      size_t n_pub = 0;
      for (size_t i = 0; i < adm.size(); ++i) {
        const AdmissionItem& a = adm[i];
        const mppi_request* r = &e->pending[a.ticket].req;
        int rc = MPPI_OK;
        if (!gates_cached_ok(e, r)) rc = MPPI_EINVAL;
        else if (!e->inst_map.contains(r->instance_id) && (int)e->inst.size() >= e->cfg.max_instances)
          rc = MPPI_EAGAIN;
        std::unique_ptr<Solve> s;
        const bool no_slot = rc == MPPI_OK && R.free_slots.empty();
        if (rc == MPPI_OK && !no_slot) rc = ring_stage(e, r, R.free_slots.back(), s);
        if (no_slot || (rc == MPPI_ENOMEM && (!R.live.empty() || n_pub > 0))) {
          // admitted by budget but not placeable yet: back to the queue
          // front until running solves release memory or slots
          e->adm->requeue_front(std::vector<AdmissionItem>(adm.begin() + i, adm.end()));
          break;
        }
        if (rc != MPPI_OK) {
          fail_ticket(e, a, rc);
          continue;
        }
        RingSolve rs;
        rs.slot = R.free_slots.back();
        R.free_slots.pop_back();
        rs.seq = R.next_seq;
        R.next_seq = R.next_seq >= 0x7FFFFFFFu ? 1u : R.next_seq + 1u;
        s->ticket = a.ticket;
        s->footprint = a.footprint;
        s->t_submit = e->ticket_submit_ns[a.ticket];
        s->t_admit = tadm;
        rs.s = std::move(s);
        ring_write_items(e, rs);
        R.live.push_back(std::move(rs));
        e->pending.erase(a.ticket);
        ++n_pub;
      }
      if (n_pub) {
        __atomic_store_n(R.ptail, R.published_p, __ATOMIC_RELEASE);
        __atomic_store_n(R.tail, R.published, __ATOMIC_RELEASE);
        e->stats.admitted += n_pub;
        e->stats.waves++;
        R.quiet_since = now;
        progress = true;
      }
      e->cv.notify_all();
    }
    if (!R.running && !R.live.empty() && !e->sticky.load()) {
      hipError_t err = launch_served(R.args, e->dw, e->cfg.T_max, e->cfg.G_max, R.max_tiles, st);
      if (err == hipSuccess) err = hipEventRecord(R.ev, st);
      if (err != hipSuccess) {
        e->sticky.store(MPPI_EDEVICE);
        e->cv.notify_all();
      } else {
        R.running = true;
        R.in_use += R.grid;   // the exit items this launch will take
        e->stats.ring_launches++;
      }
    }
    // end a quiet launch (or at destroy): its workgroups take one exit each
    if (R.running && !R.closing && R.live.empty() && (e->stop || now - R.quiet_since >= kRingQuietNs))
      ring_publish_exits(e);
    if ((!R.live.empty() || R.running) && !e->sticky.load()) {
      // poll the completion words: yield first, then short sleeps
      idle_passes = progress ? 0 : idle_passes + 1;
      lk.unlock();
      if (idle_passes < 200) std::this_thread::yield();
      else std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      idle_passes = 0;
      e->cv.wait(lk, [&] { return e->stop || e->adm->queued() > 0 || e->sticky.load(); });
      if (e->sticky.load() && !e->stop) e->cv.wait(lk, [&] { return e->stop; });
    }
  }
  // a launch still running takes its exits now (destroy synchronises the stream)
  if (R.running && !R.closing) ring_publish_exits(e);
}

// Served path.  Each pass: retire finished batches (their budget, instances
// and results are released), then admit whatever fits and launch it as one
// batch on a free serving stream.  Requests arriving while batches run are
// admitted into the next batch as memory and streams free up.
void scheduler_loop(mppi_engine* e) {
  if (e->ring.on) return scheduler_loop_ring(e);
  hipSetDevice(e->dev);
  const int nstreams = (int)e->streams.size() - 1;
  const bool timing = e->cfg.flags & MPPI_CFG_TIMING;
  std::unique_lock<std::mutex> lk(e->mu);
  while (true) {
    for (size_t i = 0; i < e->inflight.size();) {
      Inflight& b = e->inflight[i];
      const hipError_t q = hipEventQuery(b.done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) e->sticky.store(MPPI_EDEVICE);
      if (timing) add_time(e, b.t0, b.t1, true);
      const uint64_t tnow = now_ns();
      for (auto& s : b.st.solves) {
        s->t_done = tnow;
        note_result(e, s.get());
        e->adm->complete(s->footprint);
        const int st = s->res.empty() ? MPPI_EDEVICE : (int)s->res[4 * s->T + RES_STATUS];
        if (st != MPPI_OK) e->stats.failed++;
        e->stats.completed++;
      }
      release_staged(e, b.st, true);
      for (auto& s : b.st.solves) e->done[s->ticket] = std::move(s);
      for (hipEvent_t ev : {b.done, b.t0, b.t1})
        if (ev) hipEventDestroy(ev);
      e->inflight.erase(e->inflight.begin() + i);
      e->cv.notify_all();
    }
    if (e->stop && e->inflight.empty()) break;
    bool launched = false;
    if (!e->stop && !e->sticky.load() && (int)e->inflight.size() < nstreams) {
      const uint64_t cap = e->cfg.wave_queries_max ? e->cfg.wave_queries_max : (1ull << 21);
      auto adm = e->adm->admit([&](uint64_t id) {
        const int slot = e->inst_map.find(id);
        return slot >= 0 && e->inst[slot].busy;
      }, cap);
      // a request that cannot run fails on its own instead of failing the
      // batch it was admitted with: an unobserved gate without a cached
      // observation (EINVAL), or a new instance when the instance table is
      // full (EAGAIN; existing instances in the same batch still run)
      int new_slots = 0;
      for (size_t i = 0; i < adm.size();) {
        const mppi_request* r = &e->pending[adm[i].ticket].req;
        int fail = MPPI_OK;
        if (!gates_cached_ok(e, r)) {
          fail = MPPI_EINVAL;
        } else if (!e->inst_map.contains(r->instance_id)) {
          if ((int)e->inst.size() + new_slots >= e->cfg.max_instances) fail = MPPI_EAGAIN;
          else ++new_slots;
        }
        if (fail == MPPI_OK) {
          ++i;
          continue;
        }
        auto s = std::make_unique<Solve>();
        s->ticket = adm[i].ticket;
        s->T = r->T;
        s->res.assign(4 * s->T + RES_SCALARS, 0.0);
        s->res[4 * s->T + RES_STATUS] = fail;
        s->want_w = s->want_J = false;
        s->t_submit = e->ticket_submit_ns[adm[i].ticket];
        s->t_done = now_ns();
        e->adm->complete(adm[i].footprint);
        e->stats.failed++;
        e->done[adm[i].ticket] = std::move(s);
        e->pending.erase(adm[i].ticket);
        adm.erase(adm.begin() + i);
        e->cv.notify_all();
      }
      if (!adm.empty()) {
        std::vector<bool> used(nstreams + 1, false);
        for (auto& b : e->inflight) used[b.stream_idx] = true;
        int si = 1;
        while (si <= nstreams && used[si]) ++si;
        std::vector<const mppi_request*> rs;
        for (auto& a : adm) rs.push_back(&e->pending[a.ticket].req);
        Inflight b;
        b.stream_idx = si;
        const uint64_t tadm = now_ns();
        int rc = stage(e, rs, true, true, false, si, b.st);
        hipStream_t st = e->streams[si];
        if (rc == MPPI_ENOMEM && !e->inflight.empty()) {
          // admitted by budget but the pool cannot place them yet: retry once
          // a running batch has released its blocks
          e->adm->requeue_front(adm);
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(20));
          lk.lock();
          continue;
        }
        if (rc == MPPI_OK && timing) {
          hipEventCreate(&b.t0);
          hipEventCreate(&b.t1);
        }
        if (rc == MPPI_OK) rc = launch_staged(e, b.st, st, b.t0, b.t1);
        for (size_t i = 0; rc == MPPI_OK && i < b.st.solves.size(); ++i)
          rc = enqueue_fetch(e, b.st.solves[i].get(), st);
        if (rc == MPPI_OK && hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess)
          rc = dev_fail(e, hipErrorOutOfMemory);
        if (rc == MPPI_OK && hipEventRecord(b.done, st) != hipSuccess) rc = dev_fail(e, hipErrorUnknown);
        if (rc == MPPI_OK) {
          for (size_t i = 0; i < b.st.solves.size(); ++i) {
            b.st.solves[i]->ticket = adm[i].ticket;
            b.st.solves[i]->footprint = adm[i].footprint;
            b.st.solves[i]->t_submit = e->ticket_submit_ns[adm[i].ticket];
            b.st.solves[i]->t_admit = tadm;
          }
          e->stats.admitted += adm.size();
          e->stats.waves++;
          e->inflight.push_back(std::move(b));
          launched = true;
        } else {
          if (!b.st.solves.empty()) {
            hipStreamSynchronize(st);
            release_staged(e, b.st, true);
          }
          for (hipEvent_t ev : {b.done, b.t0, b.t1})
            if (ev) hipEventDestroy(ev);
          for (auto& a : adm) {
            auto s = std::make_unique<Solve>();
            s->ticket = a.ticket;
            s->T = e->pending[a.ticket].req.T;
            s->res.assign(4 * s->T + RES_SCALARS, 0.0);
            s->res[4 * s->T + RES_STATUS] = rc;
            s->want_w = s->want_J = false;
            s->t_submit = e->ticket_submit_ns[a.ticket];
            s->t_done = now_ns();
            e->adm->complete(a.footprint);
            e->stats.failed++;
            e->done[a.ticket] = std::move(s);
          }
          e->cv.notify_all();
        }
        for (auto& a : adm) e->pending.erase(a.ticket);
      }
    }
    if (launched) continue;
    if (!e->inflight.empty()) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      e->cv.wait(lk, [&] { return e->stop || e->adm->queued() > 0; });
    }
  }
}

}  // namespace
