// MPPI engine: the C ABI of include/mppi.h.
//
// Host work per solve (done in float64, then rounded once to float32):
//  - validation of the request;
//  - L = chol(Sigma) for delta u = L n (Section IV-A: delta u ~ N(0, Sigma));
//  - the latent fold c_g = W1[:, 3:] z_g + b1 (exact re-association of the
//    decoder input [p; z], Section III-B / Fig. 2);
//  - gate frames: R_g^T and the offsets of the local rollout frame, so a
//    device position dp (relative to p0 + v0 t dt) maps to the gate frame as
//    R_g^T dp + base_g(t);
//  - the rollout-independent part of the progress cost (eq. 5), which cancels
//    in the weights (eq. mppi_update) and is added back to reported costs.
// Everything else runs in the device kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
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
  int U_len;      // entries of the resident sequence that are valid
  bool busy;      // a served solve of this instance is queued or in flight
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
    z.resize((size_t)r.G * latent);
    gates.assign(r.gates, r.gates + r.G);
    for (int g = 0; g < r.G; ++g) {
      memcpy(&z[(size_t)g * latent], r.gates[g].z, sizeof(float) * latent);
      gates[g].z = &z[(size_t)g * latent];
    }
    req.gates = gates.data();
  }
};

// One solve living on the device.
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
  bool exports = false;
  uint64_t t_submit = 0, t_admit = 0, t_done = 0;
  // host result copies
  std::vector<double> res;       // 4T + RES_SCALARS
  std::vector<double> wn;        // K
  std::vector<float> J;          // K
  std::vector<float> samples, pos, sdf;
  bool want_w = false, want_J = false;
};

struct Batch {
  std::vector<std::unique_ptr<Solve>> solves;
  hipEvent_t done = nullptr;
  int stream_idx = 0;
  // fused path device arrays
  uint64_t aux_off = 0, aux_bytes = 0;
};

}  // namespace

struct mppi_engine {
  mppi_config cfg{};
  int H = 0, L = 0;
  int dev = 0;
  std::vector<hipStream_t> streams;   // [0] = blocking path; others for the served path
  bool own_stream0 = false;
  char* pool = nullptr;
  uint64_t pool_bytes = 0;
  bool own_pool = false;
  Arena arena;
  // weights
  void* wmem = nullptr;
  DeviceWeights dw{};
  std::vector<double> W0lat;   // H x latent (float32 values)
  std::vector<double> b0;      // H
  // instance table
  double* instU = nullptr;     // max_instances x T_max x 4
  uint32_t* instTick = nullptr;
  std::unordered_map<uint64_t, int> inst_map;
  std::vector<InstInfo> inst;
  std::vector<double> hover_host;   // T_max x 4, pinned copy below
  double* hover_pinned = nullptr;
  // staging for the blocking path
  char* stage = nullptr;       // pinned, max upload bytes
  uint64_t stage_bytes = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  mppi_stats stats{};
  std::atomic<int> sticky{0};
  std::mutex mu;               // guards everything above
  // served path
  std::thread sched;
  std::condition_variable cv;
  bool stop = false;
  std::unique_ptr<Admission> adm;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, OwnedRequest> pending;          // queued requests
  std::vector<Batch> inflight;
  std::unordered_map<uint64_t, std::unique_ptr<Solve>> done;   // finished, not yet polled
  std::unordered_map<uint64_t, uint64_t> ticket_submit_ns;
};

namespace {

int dev_fail(mppi_engine* e, hipError_t err) {
  if (err != hipSuccess) {
    e->sticky.store(MPPI_EDEVICE);
    return MPPI_EDEVICE;
  }
  return MPPI_OK;
}

#define HIPCHK(e, x)                                  \
  do {                                                \
    hipError_t err_ = (x);                            \
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
  const double qn = sqrt(r->x0[3] * r->x0[3] + r->x0[4] * r->x0[4] + r->x0[5] * r->x0[5] +
                         r->x0[6] * r->x0[6]);
  if (fabs(qn - 1.0) > 1e-6) return MPPI_EINVAL;
  const double w[6] = {r->Q_gate, r->Q_vis, r->Q_sdf, r->d_safe, r->R_u, 0.0};
  for (int i = 0; i < 5; ++i)
    if (std::isnan(w[i])) return MPPI_EINVAL;
  if (!isfin(r->d_safe)) return MPPI_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (!isfin(r->wp[i])) return MPPI_EINVAL;
  if (r->U_nom)
    for (int i = 0; i < 4 * r->T; ++i)
      if (!isfin(r->U_nom[i])) return MPPI_EINVAL;
  {
    if (!r->gates) return MPPI_EINVAL;
    for (int g = 0; g < r->G; ++g) {
      if (c.sdf_kind == MPPI_SDF_MLP && !r->gates[g].z) return MPPI_EINVAL;
      for (int i = 0; i < 9; ++i)
        if (!isfin(r->gates[g].R[i])) return MPPI_EINVAL;
      for (int i = 0; i < 3; ++i)
        if (!isfin(r->gates[g].t[i])) return MPPI_EINVAL;
      if (c.sdf_kind == MPPI_SDF_MLP)
        for (int i = 0; i < c.latent_dim; ++i)
          if (!std::isfinite(r->gates[g].z[i])) return MPPI_EINVAL;
    }
  }
  return cholesky4(r->Sigma, Lo);
}

// ---------------------------------------------------------------- instances
int acquire_slot(mppi_engine* e, uint64_t id, int* slot) {
  auto it = e->inst_map.find(id);
  if (it != e->inst_map.end()) {
    *slot = it->second;
    return MPPI_OK;
  }
  if ((int)e->inst.size() >= e->cfg.max_instances) return MPPI_EAGAIN;
  const int s = (int)e->inst.size();
  e->inst.push_back(InstInfo{id, e->cfg.T_max, false});
  e->inst_map[id] = s;
  // a new instance starts from hover with tick 0 (ticks were zeroed at create)
  HIPCHK(e, hipMemcpyAsync(e->instU + (size_t)s * e->cfg.T_max * 4, e->hover_pinned,
                           sizeof(double) * 4 * e->cfg.T_max, hipMemcpyHostToDevice,
                           e->streams[0]));
  HIPCHK(e, hipStreamSynchronize(e->streams[0]));
  *slot = s;
  return MPPI_OK;
}

uint64_t footprint_of(const mppi_engine* e, int K, int T, int G, bool fused) {
  const int R = fused ? fused_tile_rollouts(e->cfg.precision, e->H, G) : 1;
  const int nt = fused ? (K + R - 1) / R : 0;
  return solve_layout(K, T, G, e->H, fused, nt).total;
}

// Fill the upload part (descriptor + request data) of a solve whose device
// block starts at `base`.  Lo is the Cholesky factor from validate().
void pack_solve(mppi_engine* e, const mppi_request* r, Solve* s, const double Lo[16], char* base,
                char* host, bool fused, int tile_R) {
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
  double e_[3], vt[3];
  for (int i = 0; i < 3; ++i) {
    e_[i] = p0[i] - r->wp[i];
    vt[i] = v0[i] * tau;
    d.fprog[i] = (float)(vt[i] + e_[i]);
  }
  const double qg = r->Q_gate;
  const double c0 = vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2] +
                    2.0 * (vt[0] * e_[0] + vt[1] * e_[1] + vt[2] * e_[2]);
  d.C0 = (qg == 0.0 || c0 == 0.0) ? 0.0 : qg * c0;
  s->C0 = d.C0;
  d.hover[0] = c.mass * c.gravity;
  // nominal sequence: the request's copy, else the resident slot
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
  // gates
  float* Rt = (float*)(host + lay.Rt);
  float* bs = (float*)(host + lay.base);
  float* cf = (float*)(host + lay.cfold);
  for (int g = 0; g < G; ++g) {
    const double* R = r->gates[g].R;
    const double* tg = r->gates[g].t;
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
      for (int i = 0; i < 3; ++i) bs[((size_t)g * (T + 1) + t) * 3 + i] = (float)(o[i] + (t * r->dt) * rv[i]);
    if (c.sdf_kind == MPPI_SDF_MLP) {
      const float* z = r->gates[g].z;
      for (int m = 0; m < H; ++m) {
        double acc = e->b0[m];
        const double* wr = &e->W0lat[(size_t)m * c.latent_dim];
        for (int j = 0; j < c.latent_dim; ++j) acc += wr[j] * (double)z[j];
        cf[(size_t)g * H + m] = (float)acc;
      }
    }
  }
  float* los = (float*)(host + lay.los);
  for (int t = 0; t < T; ++t) {
    los[2 * t] = (float)(r->wp[0] - p0[0] - v0[0] * t * r->dt);
    los[2 * t + 1] = (float)(r->wp[1] - p0[1] - v0[1] * t * r->dt);
  }
  d.Rt = (const float*)(base + lay.Rt);
  d.base = (const float*)(base + lay.base);
  d.cfold = (const float*)(base + lay.cfold);
  d.los = (const float*)(base + lay.los);
  d.result = (double*)(base + lay.result);
  d.J = (float*)(base + lay.J);
  d.wn = s->want_w ? (double*)(base + lay.wn) : nullptr;
  if (!fused) {
    d.samples = (float*)(base + lay.samples);
    d.pos = (float*)(base + lay.pos);
    d.sdf = (float*)(base + lay.sdf);
    d.Jpart = (float*)(base + lay.Jpart);
    d.wt = (double*)(base + lay.wt);
  } else {
    d.partials = (double*)(base + lay.partials);
    d.tiles_done = (uint32_t*)(base + lay.tiles_done);
    d.tile_rollouts = tile_R;
    d.n_tiles = (K + tile_R - 1) / tile_R;
  }
  memcpy(host + lay.desc, &d, sizeof(SolveDesc));
  s->dt = r->dt;
  for (int i = 0; i < 3; ++i) s->v0[i] = v0[i];
}

void fill_result(mppi_engine* e, Solve* s, mppi_result* out) {
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
  if (out->weights && s->want_w) memcpy(out->weights, s->wn.data(), sizeof(double) * K);
  if (out->costs && s->want_J)
    for (int k = 0; k < K; ++k) out->costs[k] = (double)s->J[k] + s->C0;
  if (s->exports) {
    const size_t TK = (size_t)T * K, T1K = (size_t)(T + 1) * K;
    if (out->samples)
      for (int k = 0; k < K; ++k)
        for (int t = 0; t < T; ++t)
          for (int c = 0; c < 4; ++c) out->samples[((size_t)k * T + t) * 4 + c] = s->samples[c * TK + (size_t)t * K + k];
    if (out->positions)
      for (int k = 0; k < K; ++k)
        for (int t = 0; t <= T; ++t)
          for (int c = 0; c < 3; ++c)
            out->positions[((size_t)k * (T + 1) + t) * 3 + c] =
                (float)((double)s->pos[c * T1K + (size_t)t * K + k] + s->v0[c] * (t * s->dt));
    if (out->sdf)
      for (int k = 0; k < K; ++k)
        for (int t = 0; t < T; ++t) out->sdf[(size_t)k * T + t] = s->sdf[(size_t)t * K + k];
  }
  out->t_submit_ns = s->t_submit;
  out->t_admit_ns = s->t_admit;
  out->t_done_ns = s->t_done;
  (void)e;
}

// After a solve's results are on the host: instance bookkeeping.
void retire_instance(mppi_engine* e, Solve* s) {
  InstInfo& in = e->inst[s->slot];
  const int st = (int)s->res[4 * s->T + RES_STATUS];
  if (st == MPPI_OK && !(s->flags & MPPI_REQ_NO_SHIFT)) in.U_len = s->T;
  in.busy = false;
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
    HIPCHK(e, hipMemcpyAsync(s->wn.data(), base + s->lay.wn, sizeof(double) * K,
                             hipMemcpyDeviceToHost, st));
  }
  if (s->want_J) {
    s->J.resize(K);
    HIPCHK(e, hipMemcpyAsync(s->J.data(), base + s->lay.J, sizeof(float) * K,
                             hipMemcpyDeviceToHost, st));
  }
  if (s->exports) {
    s->samples.resize((size_t)4 * T * K);
    s->pos.resize((size_t)3 * (T + 1) * K);
    s->sdf.resize((size_t)T * K);
    HIPCHK(e, hipMemcpyAsync(s->samples.data(), base + s->lay.samples, 4 * s->samples.size(),
                             hipMemcpyDeviceToHost, st));
    HIPCHK(e, hipMemcpyAsync(s->pos.data(), base + s->lay.pos, 4 * s->pos.size(),
                             hipMemcpyDeviceToHost, st));
    HIPCHK(e, hipMemcpyAsync(s->sdf.data(), base + s->lay.sdf, 4 * s->sdf.size(),
                             hipMemcpyDeviceToHost, st));
  }
  return MPPI_OK;
}

// ---------------------------------------------------------------- weights
int upload_weights(mppi_engine* e, const mppi_sdf_weights* w) {
  const int H = e->H, L = e->L, D = e->cfg.latent_dim;
  const int nh = L - 1;  // hidden H x H layers
  const bool mlp = e->cfg.sdf_kind == MPPI_SDF_MLP;
  // host staging of every device array
  std::vector<float> w1p((size_t)H * 4, 0.0f), hbias((size_t)std::max(nh, 1) * H, 0.0f),
      wout(H, 0.0f);
  std::vector<float> hf32;
  std::vector<uint8_t> hlp;
  std::vector<float> wsc(std::max(nh, 1), 1.0f), asc(std::max(nh, 1), 1.0f), ainv(std::max(nh, 1), 1.0f);
  float bout = 0.0f;
  e->W0lat.assign((size_t)H * D, 0.0);
  e->b0.assign(H, 0.0);
  if (mlp) {
    for (int m = 0; m < H; ++m) {
      for (int i = 0; i < 3; ++i) w1p[m * 4 + i] = w->W[0][(size_t)m * (3 + D) + i];
      for (int j = 0; j < D; ++j) e->W0lat[(size_t)m * D + j] = w->W[0][(size_t)m * (3 + D) + 3 + j];
      e->b0[m] = w->b[0][m];
    }
    for (int l = 0; l < nh; ++l)
      for (int m = 0; m < H; ++m) hbias[(size_t)l * H + m] = w->b[l + 1][m];
    for (int m = 0; m < H; ++m) wout[m] = w->W[L][m];
    bout = w->b[L][0];
    if (e->cfg.precision == MPPI_PREC_FP32) {
      hf32.resize((size_t)nh * H * H);
      for (int l = 0; l < nh; ++l) {
        const float* W = w->W[l + 1];
        float* P = &hf32[(size_t)l * H * H];
        for (int mb = 0; mb < H / 16; ++mb)
          for (int ks = 0; ks < H / 4; ++ks)
            for (int lane = 0; lane < 64; ++lane)
              P[((size_t)mb * (H / 4) + ks) * 64 + lane] =
                  W[(size_t)(16 * mb + lane % 16) * H + 4 * ks + lane / 16];
      }
    } else {
      int rc = pack_lowp_weights(e->cfg.precision, H, L, w, hlp, wsc, asc, ainv);
      if (rc != MPPI_OK) return rc;
    }
  }
  // one device allocation for all of it
  const uint64_t o_w1p = 0;
  const uint64_t o_hb = align_up(o_w1p + 4 * w1p.size());
  const uint64_t o_wo = align_up(o_hb + 4 * hbias.size());
  const uint64_t o_hf = align_up(o_wo + 4 * wout.size());
  const uint64_t o_lp = align_up(o_hf + 4 * hf32.size());
  const uint64_t o_ws = align_up(o_lp + hlp.size());
  const uint64_t o_as = align_up(o_ws + 4 * wsc.size());
  const uint64_t o_ai = align_up(o_as + 4 * asc.size());
  const uint64_t total = align_up(o_ai + 4 * ainv.size());
  HIPCHK(e, hipMalloc(&e->wmem, total));
  char* b = (char*)e->wmem;
  HIPCHK(e, hipMemcpy(b + o_w1p, w1p.data(), 4 * w1p.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_hb, hbias.data(), 4 * hbias.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_wo, wout.data(), 4 * wout.size(), hipMemcpyHostToDevice));
  if (!hf32.empty()) HIPCHK(e, hipMemcpy(b + o_hf, hf32.data(), 4 * hf32.size(), hipMemcpyHostToDevice));
  if (!hlp.empty()) HIPCHK(e, hipMemcpy(b + o_lp, hlp.data(), hlp.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_ws, wsc.data(), 4 * wsc.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_as, asc.data(), 4 * asc.size(), hipMemcpyHostToDevice));
  HIPCHK(e, hipMemcpy(b + o_ai, ainv.data(), 4 * ainv.size(), hipMemcpyHostToDevice));
  DeviceWeights& dw = e->dw;
  dw.H = H;
  dw.n_hidden = L;
  dw.precision = e->cfg.precision;
  dw.w1p = (const float*)(b + o_w1p);
  dw.hbias = (const float*)(b + o_hb);
  dw.wout = (const float*)(b + o_wo);
  dw.bout = bout;
  dw.hidden_f32 = hf32.empty() ? nullptr : (const float*)(b + o_hf);
  dw.hidden_lp = hlp.empty() ? nullptr : (const void*)(b + o_lp);
  dw.w_scale = (const float*)(b + o_ws);
  dw.a_scale = (const float*)(b + o_as);
  dw.a_inv = (const float*)(b + o_ai);
  return MPPI_OK;
}

// ---------------------------------------------------------------- served path
void scheduler_loop(mppi_engine* e);

}  // namespace

// Prepare and launch one batch of admitted requests on stream index si.
// Caller holds e->mu.  Returns a status; on failure nothing is launched.
static int launch_batch(mppi_engine* e, std::vector<std::pair<uint64_t, OwnedRequest*>>& items,
                        int si, Batch& out);

extern "C" {

const char* mppi_status_str(int s) {
  switch (s) {
    case MPPI_OK: return "ok";
    case MPPI_PENDING: return "pending";
    case MPPI_EINVAL: return "invalid argument";
    case MPPI_ENOMEM: return "out of device memory or over the budget";
    case MPPI_EAGAIN: return "queue full or no free instance slot, retry";
    case MPPI_ENOTFOUND: return "unknown or retired ticket";
    case MPPI_ENUMERIC: return "every rollout cost is non-finite";
    case MPPI_EDEVICE: return "HIP device error";
    default: return "unknown status";
  }
}

int mppi_create(const mppi_config* cfg, const mppi_sdf_weights* w, mppi_engine** out) {
  if (!cfg || !out) return MPPI_EINVAL;
  const mppi_config& c = *cfg;
  if (c.precision < 0 || c.precision > 3 || c.path < 0 || c.path > 1 || c.sdf_kind < 0 ||
      c.sdf_kind > 1)
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
  if (c.path == MPPI_PATH_PLAIN && c.precision != MPPI_PREC_FP32) return MPPI_EINVAL;
  if (c.K_max < 1 || c.K_max > kMaxK || c.T_max < 1 || c.T_max > kMaxT || c.G_max < 1 ||
      c.G_max > kMaxG)
    return MPPI_EINVAL;
  if (c.max_instances < 1 || c.max_inflight < 1 || c.queue_depth < 1) return MPPI_EINVAL;
  if (!(c.mass > 0.0) || !isfin(c.mass) || !isfin(c.gravity)) return MPPI_EINVAL;
  for (int i = 0; i < 4; ++i)
    if (!isfin(c.u_lo[i]) || !isfin(c.u_hi[i]) || c.u_lo[i] > c.u_hi[i]) return MPPI_EINVAL;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= c.device || c.device < 0) return MPPI_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c.device) != hipSuccess) return MPPI_EDEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MPPI_EDEVICE;
  if (hipSetDevice(c.device) != hipSuccess) return MPPI_EDEVICE;

  auto e = std::make_unique<mppi_engine>();
  e->cfg = c;
  e->dev = c.device;
  e->H = c.sdf_kind == MPPI_SDF_MLP ? c.hidden : 64;
  e->L = c.sdf_kind == MPPI_SDF_MLP ? c.n_hidden : 2;
  // streams
  hipStream_t s0 = (hipStream_t)c.stream;
  if (!s0) {
    if (hipStreamCreateWithFlags(&s0, hipStreamNonBlocking) != hipSuccess) return MPPI_EDEVICE;
    e->own_stream0 = true;
  }
  e->streams.push_back(s0);
  for (int i = 0; i < 3; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return MPPI_EDEVICE;
    e->streams.push_back(s);
  }
  for (auto& ev : e->ev)
    if (hipEventCreate(&ev) != hipSuccess) return MPPI_EDEVICE;
  // weights
  int rc = upload_weights(e.get(), w);
  if (rc != MPPI_OK) return rc;
  // device pool for per-solve blocks
  if (c.device_pool) {
    e->pool = (char*)c.device_pool;
    e->pool_bytes = c.device_pool_bytes;
  } else {
    e->pool_bytes = c.hbm_budget_bytes;
    if (e->pool_bytes == 0) return MPPI_EINVAL;
    if (hipMalloc(&e->pool, e->pool_bytes) != hipSuccess) return MPPI_ENOMEM;
    e->own_pool = true;
  }
  e->arena.reset(e->pool_bytes);
  // instance table
  const size_t nI = (size_t)c.max_instances;
  if (hipMalloc(&e->instU, sizeof(double) * 4 * c.T_max * nI) != hipSuccess) return MPPI_ENOMEM;
  if (hipMalloc(&e->instTick, sizeof(uint32_t) * nI) != hipSuccess) return MPPI_ENOMEM;
  if (hipMemset(e->instTick, 0, sizeof(uint32_t) * nI) != hipSuccess) return MPPI_EDEVICE;
  if (hipHostMalloc((void**)&e->hover_pinned, sizeof(double) * 4 * c.T_max, hipHostMallocDefault) !=
      hipSuccess)
    return MPPI_ENOMEM;
  for (int t = 0; t < c.T_max; ++t) {
    e->hover_pinned[4 * t] = c.mass * c.gravity;
    e->hover_pinned[4 * t + 1] = e->hover_pinned[4 * t + 2] = e->hover_pinned[4 * t + 3] = 0.0;
  }
  // pinned staging for the blocking path
  e->stage_bytes = solve_layout(1, c.T_max, c.G_max, e->H, false, 0).upload_bytes;
  if (hipHostMalloc((void**)&e->stage, e->stage_bytes, hipHostMallocDefault) != hipSuccess)
    return MPPI_ENOMEM;
  e->stats.budget = c.hbm_budget_bytes ? c.hbm_budget_bytes : e->pool_bytes;
  e->adm = std::make_unique<Admission>(e->stats.budget, c.max_inflight, c.queue_depth);
  if (hipDeviceSynchronize() != hipSuccess) return MPPI_EDEVICE;
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
  for (auto& b : e->inflight)
    if (b.done) hipEventDestroy(b.done);
  for (auto& ev : e->ev)
    if (ev) hipEventDestroy(ev);
  for (size_t i = 0; i < e->streams.size(); ++i)
    if (i > 0 || e->own_stream0) hipStreamDestroy(e->streams[i]);
  if (e->own_pool && e->pool) hipFree(e->pool);
  if (e->wmem) hipFree(e->wmem);
  if (e->instU) hipFree(e->instU);
  if (e->instTick) hipFree(e->instTick);
  if (e->hover_pinned) hipHostFree(e->hover_pinned);
  if (e->stage) hipHostFree(e->stage);
  delete e;
  return MPPI_OK;
}

int mppi_step(mppi_engine* e, const mppi_request* r, mppi_result* out) {
  if (!e || !r || !out || !out->U_star) return MPPI_EINVAL;
  if (e->sticky.load()) return MPPI_EDEVICE;
  std::lock_guard<std::mutex> lk(e->mu);
  hipSetDevice(e->dev);
  double Lo[16];
  int rc = validate(e, r, Lo);
  if (rc != MPPI_OK) return rc;
  auto s = std::make_unique<Solve>();
  s->t_submit = now_ns();
  s->K = r->K;
  s->T = r->T;
  s->G = r->G;
  s->flags = r->flags;
  s->want_w = out->weights != nullptr;
  s->want_J = out->costs != nullptr;
  const bool fused = e->cfg.path == MPPI_PATH_FUSED;
  s->exports = !fused && (out->samples || out->positions || out->sdf);
  rc = acquire_slot(e, r->instance_id, &s->slot);
  if (rc != MPPI_OK) return rc;
  if (e->inst[s->slot].busy) return MPPI_EAGAIN;  // a served solve of this instance is pending
  if (fused) {
    // a one-solve batch through the served machinery, waited on here
    std::vector<std::pair<uint64_t, OwnedRequest*>> items;
    OwnedRequest own;
    own.take(*r, e->cfg.latent_dim);
    items.push_back({0, &own});
    Batch b;
    rc = launch_batch(e, items, 0, b);
    if (rc != MPPI_OK) return rc;
    HIPCHK(e, hipEventSynchronize(b.done));
    Solve* bs = b.solves[0].get();
    bs->t_done = now_ns();
    bs->t_submit = s->t_submit;
    bs->t_admit = s->t_submit;
    bs->want_w = s->want_w;
    fill_result(e, bs, out);
    retire_instance(e, bs);
    e->arena.release(bs->off, bs->bytes);
    if (b.aux_bytes) e->arena.release(b.aux_off, b.aux_bytes);
    hipEventDestroy(b.done);
    e->stats.completed++;
    return out->status;
  }
  s->lay = solve_layout(r->K, r->T, r->G, e->H, false, 0);
  s->bytes = s->lay.total;
  if (!e->arena.alloc(s->bytes, &s->off)) return MPPI_ENOMEM;
  char* base = e->pool + s->off;
  pack_solve(e, r, s.get(), Lo, base, e->stage, false, 1);
  hipStream_t st = e->streams[0];
  const bool timing = e->cfg.flags & MPPI_CFG_TIMING;
  auto fail = [&](hipError_t err) {
    e->arena.release(s->off, s->bytes);
    return dev_fail(e, err);
  };
  hipError_t err = hipMemcpyAsync(base, e->stage, s->lay.upload_bytes, hipMemcpyHostToDevice, st);
  if (err != hipSuccess) return fail(err);
  if (timing) hipEventRecord(e->ev[2], st);
  PlainShape shp{r->K, r->T, r->G, e->cfg.sdf_kind};
  err = launch_plain((const SolveDesc*)(base + s->lay.desc), shp, e->dw, st,
                     timing ? e->ev[0] : nullptr, timing ? e->ev[1] : nullptr);
  if (err != hipSuccess) return fail(err);
  if (timing) hipEventRecord(e->ev[3], st);
  rc = enqueue_fetch(e, s.get(), st);
  if (rc != MPPI_OK) {
    e->arena.release(s->off, s->bytes);
    return rc;
  }
  err = hipStreamSynchronize(st);
  if (err != hipSuccess) return fail(err);
  s->t_admit = s->t_submit;
  s->t_done = now_ns();
  if (timing) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e->ev[0], e->ev[1]) == hipSuccess) {
      e->stats.sdf_ms += ms;
      e->stats.sdf_launches++;
    }
    if (hipEventElapsedTime(&ms, e->ev[2], e->ev[3]) == hipSuccess) {
      e->stats.solve_ms += ms;
      e->stats.solve_launches++;
    }
  }
  fill_result(e, s.get(), out);
  retire_instance(e, s.get());
  e->arena.release(s->off, s->bytes);
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
  const bool fused = e->cfg.path == MPPI_PATH_FUSED;
  const uint64_t fp = footprint_of(e, r->K, r->T, r->G, fused);
  const uint64_t t = e->next_ticket;
  rc = e->adm->push(AdmissionItem{t, r->instance_id, fp});
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
  Solve* s = it->second.get();
  if (!out->U_star) return MPPI_EINVAL;
  fill_result(e, s, out);
  const int st = out->status;
  e->done.erase(it);
  e->ticket_submit_ns.erase(ticket);
  return st;
}

int mppi_drain(mppi_engine* e) {
  if (!e) return MPPI_EINVAL;
  std::unique_lock<std::mutex> lk(e->mu);
  e->cv.wait(lk, [&] {
    return e->sticky.load() != 0 || (e->adm->queued() == 0 && e->inflight.empty());
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
  return footprint_of(e, K, T, G, e->cfg.path == MPPI_PATH_FUSED);
}

}  // extern "C"

// ---------------------------------------------------------------- batches
static int launch_batch(mppi_engine* e, std::vector<std::pair<uint64_t, OwnedRequest*>>& items,
                        int si, Batch& out) {
  const bool fused = e->cfg.path == MPPI_PATH_FUSED;
  hipStream_t st = e->streams[si];
  out.stream_idx = si;
  std::vector<std::unique_ptr<Solve>> solves;
  std::vector<char> host;
  auto release_all = [&]() {
    for (auto& s : solves) e->arena.release(s->off, s->bytes);
    if (out.aux_bytes) e->arena.release(out.aux_off, out.aux_bytes);
    out.aux_bytes = 0;
  };
  int total_tiles = 0;
  std::vector<int2> tiles;
  for (auto& it : items) {
    const mppi_request* r = &it.second->req;
    double Lo[16];
    int rc = validate(e, r, Lo);
    auto s = std::make_unique<Solve>();
    s->ticket = it.first;
    s->K = r->K;
    s->T = r->T;
    s->G = r->G;
    s->flags = r->flags;
    s->want_w = true;
    s->want_J = true;
    if (rc == MPPI_OK) rc = acquire_slot(e, r->instance_id, &s->slot);
    if (rc != MPPI_OK) {
      release_all();
      return rc;
    }
    const int R = fused ? fused_tile_rollouts(e->cfg.precision, e->H, r->G) : 1;
    const int nt = fused ? (r->K + R - 1) / R : 0;
    s->lay = solve_layout(r->K, r->T, r->G, e->H, fused, nt);
    s->bytes = s->lay.total;
    if (!e->arena.alloc(s->bytes, &s->off)) {
      release_all();
      return MPPI_ENOMEM;
    }
    host.assign(s->lay.upload_bytes, 0);
    char* base = e->pool + s->off;
    pack_solve(e, r, s.get(), Lo, base, host.data(), fused, R);
    // The copy is synchronous from pageable memory into the device block
    // before any kernel of this batch is enqueued.
    hipError_t err = hipMemcpyAsync(base, host.data(), s->lay.upload_bytes, hipMemcpyHostToDevice, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) {
      release_all();
      return dev_fail(e, err);
    }
    if (fused) {
      for (int i = 0; i < nt; ++i) tiles.push_back(int2{(int)solves.size(), i * R});
      total_tiles += nt;
    }
    e->inst[s->slot].busy = true;
    solves.push_back(std::move(s));
  }
  const bool timing = e->cfg.flags & MPPI_CFG_TIMING;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (timing) {
    hipEventCreate(&t0);
    hipEventCreate(&t1);
  }
  if (!fused) {
    for (auto& s : solves) {
      PlainShape shp{s->K, s->T, s->G, e->cfg.sdf_kind};
      hipError_t err = launch_plain((const SolveDesc*)(e->pool + s->off + s->lay.desc), shp, e->dw,
                                    st, timing ? t0 : nullptr, timing ? t1 : nullptr);
      if (err != hipSuccess) {
        release_all();
        return dev_fail(e, err);
      }
    }
  } else {
    // descriptor array + tile list + work counter in one aux block
    const size_t nS = solves.size();
    out.aux_bytes = align_up(sizeof(SolveDesc) * nS) + align_up(sizeof(int2) * tiles.size()) + 256;
    if (!e->arena.alloc(out.aux_bytes, &out.aux_off)) {
      out.aux_bytes = 0;
      release_all();
      return MPPI_ENOMEM;
    }
    // longest tiles first (work per tile grows with T and G)
    std::stable_sort(tiles.begin(), tiles.end(), [&](const int2& a, const int2& b) {
      const Solve* sa = solves[a.x].get();
      const Solve* sb = solves[b.x].get();
      return sa->T * sa->G > sb->T * sb->G;
    });
    std::vector<char> aux(out.aux_bytes, 0);
    for (size_t i = 0; i < nS; ++i) memcpy(aux.data() + i * sizeof(SolveDesc), &solves[i]->desc, sizeof(SolveDesc));
    const uint64_t o_tiles = align_up(sizeof(SolveDesc) * nS);
    memcpy(aux.data() + o_tiles, tiles.data(), sizeof(int2) * tiles.size());
    const uint64_t o_cnt = o_tiles + align_up(sizeof(int2) * tiles.size());
    char* ab = e->pool + out.aux_off;
    hipError_t err = hipMemcpyAsync(ab, aux.data(), out.aux_bytes, hipMemcpyHostToDevice, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) {
      release_all();
      return dev_fail(e, err);
    }
    int maxT = 1;
    for (auto& s : solves) maxT = std::max(maxT, s->T);
    FusedBatch fb{(const SolveDesc*)ab, (const int2*)(ab + o_tiles), (int)tiles.size(),
                  (uint32_t*)(ab + o_cnt)};
    err = launch_fused(fb, e->dw, maxT, st, timing ? t0 : nullptr, timing ? t1 : nullptr);
    if (err != hipSuccess) {
      release_all();
      return dev_fail(e, err);
    }
  }
  for (auto& s : solves) {
    int rc = enqueue_fetch(e, s.get(), st);
    if (rc != MPPI_OK) {
      release_all();
      return rc;
    }
  }
  hipError_t err = hipEventCreateWithFlags(&out.done, hipEventDisableTiming);
  if (err == hipSuccess) err = hipEventRecord(out.done, st);
  if (err != hipSuccess) {
    release_all();
    return dev_fail(e, err);
  }
  if (timing) {
    hipEventSynchronize(t1);
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, t0, t1) == hipSuccess) {
      e->stats.sdf_ms += ms;
      e->stats.sdf_launches++;
    }
    hipEventDestroy(t0);
    hipEventDestroy(t1);
  }
  e->stats.waves++;
  out.solves = std::move(solves);
  (void)total_tiles;
  return MPPI_OK;
}

namespace {

// Served path: admit, batch, launch, complete.  One batch per free stream;
// requests that arrive while batches run are admitted into the next batch.
void scheduler_loop(mppi_engine* e) {
  hipSetDevice(e->dev);
  const int nstreams = (int)e->streams.size() - 1;   // streams 1.. for serving
  std::unique_lock<std::mutex> lk(e->mu);
  while (true) {
    // 1. retire finished batches
    for (size_t i = 0; i < e->inflight.size();) {
      Batch& b = e->inflight[i];
      hipError_t q = hipEventQuery(b.done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) e->sticky.store(MPPI_EDEVICE);
      const uint64_t tnow = now_ns();
      for (auto& s : b.solves) {
        s->t_done = tnow;
        retire_instance(e, s.get());
        e->arena.release(s->off, s->bytes);
        e->adm->complete(s->footprint);
        const int st = s->res.empty() ? MPPI_EDEVICE : (int)s->res[4 * s->T + RES_STATUS];
        if (st != MPPI_OK) e->stats.failed++;
        e->stats.completed++;
        e->done[s->ticket] = std::move(s);
      }
      if (b.aux_bytes) e->arena.release(b.aux_off, b.aux_bytes);
      hipEventDestroy(b.done);
      e->inflight.erase(e->inflight.begin() + i);
      e->cv.notify_all();
    }
    if (e->stop && e->inflight.empty()) break;
    // 2. admit and launch while a serving stream is free
    bool launched = false;
    if (!e->stop && !e->sticky.load() && (int)e->inflight.size() < nstreams) {
      auto adm = e->adm->admit([&](uint64_t id) {
        auto it = e->inst_map.find(id);
        return it != e->inst_map.end() && e->inst[it->second].busy;
      });
      if (!adm.empty()) {
        std::vector<bool> used(nstreams + 1, false);
        for (auto& b : e->inflight) used[b.stream_idx] = true;
        int si = 1;
        while (si <= nstreams && used[si]) ++si;
        std::vector<std::pair<uint64_t, OwnedRequest*>> items;
        for (auto& a : adm) items.push_back({a.ticket, &e->pending[a.ticket]});
        Batch b;
        const uint64_t tadm = now_ns();
        int rc = launch_batch(e, items, si, b);
        if (rc == MPPI_OK) {
          for (size_t i = 0; i < b.solves.size(); ++i) {
            b.solves[i]->footprint = adm[i].footprint;
            b.solves[i]->t_submit = e->ticket_submit_ns[adm[i].ticket];
            b.solves[i]->t_admit = tadm;
          }
          e->stats.admitted += adm.size();
          e->inflight.push_back(std::move(b));
          launched = true;
        } else {
          // fail these requests with the status; their budget is returned
          for (auto& a : adm) {
            auto s = std::make_unique<Solve>();
            s->ticket = a.ticket;
            s->T = e->pending[a.ticket].req.T;
            s->res.assign(4 * s->T + RES_SCALARS, 0.0);
            s->res[4 * s->T + RES_STATUS] = rc;
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
      // poll the running batches without holding the lock for long
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      e->cv.wait(lk, [&] { return e->stop || e->adm->queued() > 0; });
    }
  }
}

}  // namespace
