// C ABI of the library (declared in include/lb.h): handle lifetime, argument
// checking, buffer ownership, the step loop and the field/diagnostic copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lb.h"
#include "diag_kernels.hpp"
#include "engine.hpp"
#include "llb_kernels.hpp"
#include "mlp_kernels.hpp"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(LB_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                      __FILE__, __LINE__);                                   \
  } while (0)

const LatticeOps* ops_for(int lattice) {
  switch (lattice) {
    case LB_D2Q9: return ops_d2q9();
    case LB_D3Q19: return ops_d3q19();
    case LB_D3Q27: return ops_d3q27();
  }
  return nullptr;
}

const LlbOps* llb_for(int lattice) {
  switch (lattice) {
    case LB_D2Q9: return llb_d2q9();
    case LB_D3Q19: return llb_d3q19();
    case LB_D3Q27: return llb_d3q27();
  }
  return nullptr;
}

const InPlaceOps* inplace_for(int lattice) {
  switch (lattice) {
    case LB_D2Q9: return inplace_d2q9();
    case LB_D3Q19: return inplace_d3q19();
    case LB_D3Q27: return inplace_d3q27();
  }
  return nullptr;
}

size_t storage_bytes(int st) {
  switch (st) {
    case LB_F64: return 8;
    case LB_F32:
    case LB_F32_TOTAL:
    case LB_F32_SHIFTED: return 4;
    case LB_F16_SHIFTED:
    case LB_BF16_SHIFTED:
    case LB_F16_TOTAL:
    case LB_BF16_TOTAL:
    case LB_F16C_TOTAL: return 2;
  }
  return 0;
}

bool total_layout(int st) {
  return st == LB_F32_TOTAL || st == LB_F16_TOTAL || st == LB_BF16_TOTAL || st == LB_F16C_TOTAL;
}

}  // namespace

struct lb_handle {
  lb_params p;
  const LatticeOps* ops = nullptr;
  int q = 0, d = 0;
  uint32_t N = 0;
  size_t esize = 0;  // bytes per stored population
  // population planes: rows of px >= nx sites, NF = px ny nz elements per
  // plane (the read-once two-copy step pads rows of 4- and 8-byte
  // populations to a multiple of 128 bytes; the padding is never read)
  uint32_t px = 0;
  size_t NF = 0;
  // stride of the per-site planes of the total layout's scalars and of the
  // read-once partial sums P (N rounded up to 64 sites, plus 64)
  size_t NS = 0;
  size_t rsize = 0;  // bytes per field value (8 for FP64, else 4)
  hipStream_t stream = nullptr;
  int device = 0;
  void* f[2] = {nullptr, nullptr};
  float* sc[2] = {nullptr, nullptr};  // recolouring scalars (total layout only)
  bool total = false;
  int cur = 0;
  // in-place streaming: one copy f[0] (and sc[0]); ip_odd says which kind of
  // step comes next (0: even, from the canonical layout)
  const InPlaceOps* ip = nullptr;
  int ip_odd = 0;
  bool in_place() const { return ip != nullptr; }
  // moment-based scheme: f[0] / f[1] hold the 15 moments per site, W the 11
  // pre-collision moments between the two passes
  const LlbOps* llb = nullptr;
  void* W = nullptr;
  bool moments() const { return llb != nullptr; }
  // phase field: two buffers.  phi_at(pcur) is what the next collision pass
  // reads; phi_at(pfield) belongs to the fields of the last step (or of the
  // initial state).  The read-once step's combine pass writes the other buffer.
  void* phi = nullptr;
  void* phi2 = nullptr;
  int pcur = 0, pfield = 0;
  void* phi_at(int k) const { return k ? phi2 : phi; }
  void* phi_field() const { return phi_at(pfield); }
  // read-once step (lb_params.phase_pass, lb_phase_mode): the collision
  // pass scatters the next step's colour densities into ro_part (2 x NS) and
  // ro_halo (per tile-march halo blocks, marches of ro_zb planes); phi_ready
  // says that phi_at(pcur) already holds the phase field of the next pull
  bool ro = false;
  bool phi_ready = false;
  int ro_zb = 1;
  void* ro_part = nullptr;
  void* ro_halo = nullptr;
  size_t ro_halo_bytes = 0;
  void* rho_a = nullptr;
  void* rho_b = nullptr;
  void* u = nullptr;
  void* fnc = nullptr;
  uint8_t* flags = nullptr;
  int32_t* labels = nullptr;
  double* diag_partial = nullptr;
  double* diag_out = nullptr;
  unsigned int* ccl_count = nullptr;
  double* drops = nullptr;
  int drops_cap = 0;
  long long t = 0;
  bool initialised = false;
  bool fields_valid = false;  // macroscopic fields describe the current state
  int z_per_block = 1;
  // ensemble of independent channels (n_channels > 1): each channel is a
  // full single-lattice handle sharing this handle's stream; a batched step
  // is one phase launch and one collision launch over all channels' tiles
  std::vector<lb_handle*> chans;
  ChannelDev* d_chans = nullptr;
  uint32_t* d_items_ph = nullptr;    // phase tiles of every channel
  uint32_t* d_items_co = nullptr;    // collision tiles of every channel
  uint32_t* d_items_cb = nullptr;    // read-once step: combine blocks of every channel
  uint32_t n_items_ph = 0, n_items_co = 0, n_items_cb = 0;
  lb_tuning tune{};                  // ensemble launch configuration
  // read-once batched collision: store the populations through L2 (some
  // channel's population rows do not start on 64-byte boundaries, so
  // neighbouring tiles write the two ends of one line; non-temporal stores
  // would send each part to memory on its own)
  bool ens_cached = false;
  hipGraphExec_t graph = nullptr;    // two non-field steps (ensemble: parity 0 then 1)
  int graph_key = 0;                 // single lattice: the parities it was captured at
  bool ensemble() const { return !chans.empty(); }
  // learned near-contact closure: FP32 parameters, Adam moments, training
  // scratch, input ranges and the network in MFMA operand order
  float* mlp_theta = nullptr;
  float* mlp_m1 = nullptr;
  float* mlp_m2 = nullptr;
  float* mlp_grad = nullptr;
  float* mlp_part = nullptr;         // partial gradients, mlp_part_cap workgroups
  float* mlp_part_l = nullptr;
  int mlp_part_cap = 0;
  float* mlp_lo = nullptr;           // [32] lo, then [32] hi
  uint32_t* mlp_bad = nullptr;
  MlpPacked* mlp_net = nullptr;
  float mlp_gmin = INFINITY;
  bool mlp_weights = false;
  // per-kernel timing: hipEvent pairs recorded on the handle's stream around
  // each launch while profiling is on
  bool prof_on = false;
  std::vector<hipEvent_t> prof_events;
  std::vector<int> prof_kind;  // one entry per event pair: 0 phase, 1 collide, 2 combine
  size_t prof_used = 0;

  StepArgs step_args() const {
    StepArgs a{};
    a.nx = p.nx; a.ny = p.ny; a.nz = p.nz;
    a.wall_x = p.wall[0]; a.wall_y = p.wall[1]; a.wall_z = p.wall[2];
    a.N = N;
    a.px = px;
    a.NF = (uint32_t)NF;
    a.NS = (uint32_t)NS;
    a.QN = (uint64_t)q * NF;
    a.omega = 1.0 / p.tau;
    a.guo = 1.0 - 0.5 / p.tau;
    a.visc_mix = p.tau_b != 0.0 && p.tau_b != p.tau;
    a.inv_nu_a = 3.0 / (p.tau - 0.5);
    a.inv_nu_b = a.visc_mix ? 3.0 / (p.tau_b - 0.5) : a.inv_nu_a;
    a.A = p.A;
    a.beta = p.beta;
    a.half_rho0 = 0.5 * p.rho0;
    a.fx = p.body_force[0]; a.fy = p.body_force[1]; a.fz = p.body_force[2];
    a.nc_A = p.nc_A;
    a.nc_hmin = p.nc_hmin;
    a.nc_steps = (int)std::floor(p.nc_hmax);
    a.phi_I = p.phi_interface;
    a.z_per_block = z_per_block;
    a.sround = p.rounding == LB_ROUND_STOCHASTIC;
    a.step = 0;
    return a;
  }
  FieldPtrs field_ptrs() const { return FieldPtrs{rho_a, rho_b, u, fnc, flags}; }
};

extern "C" {

void lb_params_default(lb_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->lattice = LB_D3Q27;
  p->storage = LB_F32;
  p->nc_mode = LB_NC_OFF;
  p->nx = p->ny = p->nz = 64;
  p->tau = 1.0;
  p->A = 0.01;
  p->beta = 0.7;
  p->rho0 = 1.0;
  p->nc_A = 0.02;
  p->nc_hmin = 2.0;
  p->nc_hmax = 3.0;
  p->phi_interface = 0.9;
}

const char* lb_error_string(int code) {
  switch (code) {
    case LB_OK: return "ok";
    case LB_EINVAL: return "invalid argument";
    case LB_ENOMEM: return "out of device memory";
    case LB_EHIP: return "HIP runtime error";
    case LB_ENUMERIC: return "numerical watchdog tripped (NaN/Inf, rho <= 0 or |u| > 0.3)";
    case LB_ENODEV: return "no HIP device";
    case LB_EUNSUPPORTED: return "not supported by this build";
  }
  return "unknown status";
}

const char* lb_last_error(void) { return g_err.c_str(); }

int lb_lattice_table(int lattice, int* q, int* c, double* w, int* opp, double* B) {
  auto fill = [&](auto L) -> int {
    using Lt = decltype(L);
    if (q) *q = Lt::Q;
    for (int i = 0; i < Lt::Q; ++i) {
      if (c) { c[3 * i] = Lt::cx[i]; c[3 * i + 1] = Lt::cy[i]; c[3 * i + 2] = Lt::cz[i]; }
      if (w) w[i] = Lt::w[i];
      if (opp) opp[i] = Lt::opp[i];
      if (B) B[i] = B_coef<Lt>(i);
    }
    return LB_OK;
  };
  switch (lattice) {
    case LB_D2Q9: return fill(D2Q9{});
    case LB_D3Q19: return fill(D3Q19{});
    case LB_D3Q27: return fill(D3Q27{});
  }
  return fail(LB_EINVAL, "unknown lattice %d", lattice);
}

static int validate(const lb_params* p) {
  if (!p) return fail(LB_EINVAL, "params is NULL");
  if (!ops_for(p->lattice)) return fail(LB_EINVAL, "unknown lattice %d", p->lattice);
  if (storage_bytes(p->storage) == 0) return fail(LB_EINVAL, "unknown storage %d", p->storage);
  if (p->nc_mode != LB_NC_OFF && p->nc_mode != LB_NC_EXPLICIT && p->nc_mode != LB_NC_MLP)
    return fail(LB_EINVAL, "unknown nc_mode %d", p->nc_mode);
  if (p->nc_mode == LB_NC_MLP && (p->lattice == LB_D2Q9 || !mlp_storage(p->storage)))
    return fail(LB_EINVAL, "the learned closure needs a 3D lattice and storage LB_F64, LB_F32 or a total layout");
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return fail(LB_EINVAL, "sizes must be positive");
  if (p->lattice == LB_D2Q9 && (p->nz != 1 || p->wall[2])) return fail(LB_EINVAL, "D2Q9 needs nz == 1 and no z wall");
  if (p->lattice == LB_D2Q9 && (p->body_force[2] != 0.0 || p->u0[2] != 0.0))
    return fail(LB_EINVAL, "D2Q9 needs zero z components of body_force and u0");
  for (int a = 0; a < 3; ++a)
    if (p->wall[a] != 0 && p->wall[a] != 1) return fail(LB_EINVAL, "wall[%d] must be 0 or 1", a);
  const double N = (double)p->nx * p->ny * p->nz;
  // a pulled population is addressed within the planes of its velocity pair
  // {i, opp(i)} with a 32-bit byte offset: 2 planes in 3D, up to 3 in D2Q9
  const double span = p->lattice == LB_D2Q9 ? 3.0 : 2.0;
  if (N * span * storage_bytes(p->storage) > 4294967295.0)
    return fail(LB_EINVAL, "%.0f sites x %d bytes: the planes of one velocity pair (%.0f bytes) must stay "
                "below 4 GiB (32-bit lane offsets)", N, storage_bytes(p->storage),
                N * span * storage_bytes(p->storage));
  if (N > 2147483647.0) return fail(LB_EINVAL, "at most 2^31 - 1 sites (droplet labels are int32)");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LB_EINVAL, "tau must exceed 1/2");
  if (p->tau_b != 0.0 && (!(p->tau_b > 0.5) || !std::isfinite(p->tau_b)))
    return fail(LB_EINVAL, "tau_b must exceed 1/2 (or be 0 for one viscosity)");
  if (!(p->rho0 > 0.0)) return fail(LB_EINVAL, "rho0 must be positive");
  if (!(p->phi_interface > 0.0 && p->phi_interface < 1.0)) return fail(LB_EINVAL, "phi_interface must lie in (0,1)");
  if (!std::isfinite(p->A) || !std::isfinite(p->beta)) return fail(LB_EINVAL, "A and beta must be finite");
  if (p->nc_mode != LB_NC_OFF) {
    // the near-contact stencil reaches 4 sites; each axis must be at least that long
    if (p->nx < 4 || p->ny < 4 || (p->lattice != LB_D2Q9 && p->nz < 4))
      return fail(LB_EINVAL, "near contact needs every axis >= 4 sites");
    if (!(p->nc_hmax >= 1.0 && p->nc_hmax < 4.0)) return fail(LB_EINVAL, "nc_hmax must lie in [1, 4)");
    if (!(p->nc_hmin > 0.0)) return fail(LB_EINVAL, "nc_hmin must be positive");
  }
  if (p->diag_every < 0) return fail(LB_EINVAL, "diag_every must be >= 0");
  if (p->streaming != LB_STREAM_TWO_COPIES && p->streaming != LB_STREAM_IN_PLACE)
    return fail(LB_EINVAL, "unknown streaming %d", p->streaming);
  if (p->scheme != LB_SCHEME_POPULATIONS && p->scheme != LB_SCHEME_MOMENTS)
    return fail(LB_EINVAL, "unknown scheme %d", p->scheme);
  if (p->scheme == LB_SCHEME_MOMENTS) {
    if (p->storage != LB_F64 && p->storage != LB_F32)
      return fail(LB_EINVAL, "the moment-based scheme stores its moments in LB_F64 or LB_F32");
    if (p->nc_mode == LB_NC_MLP) return fail(LB_EINVAL, "the moment-based scheme takes nc_mode off or explicit");
    if (p->streaming != LB_STREAM_TWO_COPIES) return fail(LB_EINVAL, "the moment-based scheme streams with two copies");
  }
  if (p->phase_pass != LB_PHASE_AUTO && p->phase_pass != LB_PHASE_SCATTER && p->phase_pass != LB_PHASE_PASS)
    return fail(LB_EINVAL, "unknown phase_pass %d", p->phase_pass);
  if (p->rounding != LB_ROUND_NEAREST && p->rounding != LB_ROUND_STOCHASTIC)
    return fail(LB_EINVAL, "unknown rounding %d", p->rounding);
  if (p->rounding == LB_ROUND_STOCHASTIC && p->storage != LB_F16_TOTAL && p->storage != LB_BF16_TOTAL)
    return fail(LB_EINVAL, "stochastic rounding applies to LB_F16_TOTAL and LB_BF16_TOTAL only");
  if (p->rounding == LB_ROUND_STOCHASTIC && p->nc_mode == LB_NC_MLP)
    return fail(LB_EINVAL, "stochastic rounding takes nc_mode off or explicit");
  return LB_OK;
}

int lb_destroy(lb_handle* h) {
  if (!h) return LB_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  for (lb_handle* c : h->chans) lb_destroy(c);
  h->chans.clear();
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  for (void* b : {(void*)h->d_chans, (void*)h->d_items_ph, (void*)h->d_items_co, (void*)h->d_items_cb})
    if (b) (void)hipFree(b);
  for (hipEvent_t e : h->prof_events) (void)hipEventDestroy(e);
  void* bufs[] = {h->f[0], h->f[1], h->sc[0], h->sc[1], h->W, h->phi, h->phi2, h->ro_part, h->ro_halo, h->rho_a, h->rho_b, h->u, h->fnc, h->flags, h->labels,
                  h->diag_partial, h->diag_out, h->ccl_count, h->drops, h->mlp_theta, h->mlp_m1, h->mlp_m2,
                  h->mlp_grad, h->mlp_part, h->mlp_part_l, h->mlp_lo, h->mlp_bad, h->mlp_net};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  (void)hipSetDevice(dev);
  delete h;
  return LB_OK;
}

static int dev_alloc(void** p, size_t bytes, const char* what) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EHIP, "hipMalloc(%s, %zu bytes): %s", what, bytes,
                hipGetErrorString(e));
  }
  return LB_OK;
}

static int create_single(const lb_params* p, void* hip_stream, lb_handle** out, bool channel = false);
static int ensemble_plan(lb_handle* h);
static int ro_plan(lb_handle* h);

int lb_create(const lb_params* p, int n_channels, void* hip_stream, lb_handle** out) {
  if (!out) return fail(LB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return fail(LB_EINVAL, "params is NULL");
  if (n_channels < 1 || n_channels > (int)ITEM_CH_MASK + 1)
    return fail(LB_EINVAL, "n_channels must lie in [1, %u] (got %d)", ITEM_CH_MASK + 1, n_channels);
  for (int c = 0; c < n_channels; ++c) {
    int rc = validate(&p[c]);
    if (rc) return rc;
    if (p[c].lattice != p[0].lattice || p[c].storage != p[0].storage || p[c].nc_mode != p[0].nc_mode)
      return fail(LB_EINVAL, "channel %d: lattice, storage and nc_mode must agree across channels", c);
  }
  if (n_channels == 1) return create_single(p, hip_stream, out);
  for (int c = 0; c < n_channels; ++c) {
    if (p[c].streaming != LB_STREAM_TWO_COPIES)
      return fail(LB_EINVAL, "channel %d: ensembles stream with two copies (LB_STREAM_TWO_COPIES)", c);
    if (p[c].scheme != LB_SCHEME_POPULATIONS)
      return fail(LB_EINVAL, "channel %d: ensembles use the population scheme", c);
    if (p[c].rounding != LB_ROUND_NEAREST)
      return fail(LB_EINVAL, "channel %d: ensembles round to nearest (stochastic rounding is single-lattice)", c);
    if (p[c].phase_pass != p[0].phase_pass)
      return fail(LB_EINVAL, "channel %d: phase_pass must agree across channels", c);
  }
  if (p[0].nc_mode == LB_NC_MLP) return fail(LB_EINVAL, "ensembles take nc_mode LB_NC_OFF or LB_NC_EXPLICIT");
  if (!ensemble_storage(p[0].storage))
    return fail(LB_EINVAL, "ensembles take storage LB_F64, LB_F32 or a total layout (got %d)", p[0].storage);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(LB_ENODEV, "no HIP device");
  }
  lb_handle* h = new lb_handle();
  h->p = p[0];
  h->ops = ops_for(p[0].lattice);
  h->q = h->ops->q;
  h->d = h->ops->d;
  h->esize = storage_bytes(p[0].storage);
  h->rsize = p[0].storage == LB_F64 ? 8 : 4;
  h->total = total_layout(p[0].storage);
  h->stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&h->device);
  for (int c = 0; c < n_channels; ++c) {
    lb_handle* sub = nullptr;
    int rc = create_single(&p[c], hip_stream, &sub, true);
    if (rc) { lb_destroy(h); return rc; }
    h->chans.push_back(sub);
    h->N += sub->N;
  }
  h->ro = h->chans[0]->ro;
  h->tune.mode = LB_ENSEMBLE_BATCHED;
  h->tune.z_per_block = 4;
  h->tune.use_graph = 1;
  int rc = ensemble_plan(h);
  if (rc) { lb_destroy(h); return rc; }
  *out = h;
  g_err.clear();
  return LB_OK;
}

// channel: a channel of an ensemble (stepped by the ensemble's launches)
static int create_single(const lb_params* p, void* hip_stream, lb_handle** out, bool channel) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(LB_ENODEV, "no HIP device");
  }
  lb_handle* h = new lb_handle();
  h->p = *p;
  h->ops = ops_for(p->lattice);
  h->q = h->ops->q;
  h->d = h->ops->d;
  h->N = (uint32_t)((size_t)p->nx * p->ny * p->nz);
  h->esize = storage_bytes(p->storage);
  h->rsize = p->storage == LB_F64 ? 8 : 4;
  h->total = total_layout(p->storage);
  h->stream = (hipStream_t)hip_stream;
  if (p->streaming == LB_STREAM_IN_PLACE) h->ip = inplace_for(p->lattice);
  if (p->scheme == LB_SCHEME_MOMENTS) h->llb = llb_for(p->lattice);
  (void)hipGetDevice(&h->device);
  // tiles march through z; aim for about 1024 workgroups (4 per CU): longer
  // marches amortise the staging of the first planes, measured best at 16
  // planes on the 256 x 128 x 128 channel (FP16 total layout +2%, moment
  // scheme +6% over 8 planes; plain FP32 unchanged)
  {
    const long bxy = (long)((p->nx + TILE_X - 1) / TILE_X) * ((p->ny + TILE_Y - 1) / TILE_Y);
    long zb = (bxy * p->nz) / 1024;
    if (zb < 1) zb = 1;
    if (zb > 16) zb = 16;
    if (zb > p->nz) zb = p->nz;
    if (const char* env = std::getenv("LB_Z_PER_BLOCK")) {
      const long v = std::atol(env);
      if (v >= 1) zb = v;
    }
    h->z_per_block = (int)zb;
  }
  const size_t N = h->N;
  {
    const bool total16 = p->storage == LB_F16_TOTAL || p->storage == LB_BF16_TOTAL || p->storage == LB_F16C_TOTAL;
    const int mode = p->phase_pass == LB_PHASE_AUTO ? (total16 ? LB_PHASE_PASS : LB_PHASE_SCATTER) : p->phase_pass;
    h->ro = !h->moments() && mode == LB_PHASE_SCATTER;
  }
  // Row pitch of the population planes.  Rows whose length is not a multiple
  // of 128 bytes start inside a cache line, so a wave's loads and stores
  // touch an extra line and the line at a row end is written in two parts
  // by neighbouring tiles.  Measured: ensembles of 96 D3Q19 channels (FP32),
  // 100 x 80 x 80 channels at 2.4 TB/s against 4.0-5.0 TB/s for 96-, 112-,
  // 128- and 160-wide ones; a 250 x 128 x 128 channel at 5829 (FP32
  // read-once), 5014 (FP32 two-pass) and 12502 MLUPS (FP16 total) with
  // unpadded rows, 9633, 7455 and 17889 with padded ones.  Every population
  // layout pads each row to the next multiple of 128 bytes.  The pad sites
  // are never read (pulls wrap at nx); in the read-once two-copy step the
  // lanes in the padding store into it, so that a row's last line is written
  // whole.  The moment scheme keeps plain rows: its passes are bound by
  // issue, and padded rows measured 2% slower (250 x 128 x 128, FP32:
  // 13134 against 13404 MLUPS); its kernels index the moment planes with px
  // all the same.
  h->px = (uint32_t)p->nx;
  const char* row_env = std::getenv("LB_ROW_PAD");  // measurement override: "0" keeps px = nx
  if (!(row_env && !std::strcmp(row_env, "0")) && !h->moments()) {
    const uint32_t m = (uint32_t)(128 / h->esize);
    const uint32_t px = ((uint32_t)p->nx + m - 1) / m * m;
    const double span = p->lattice == LB_D2Q9 ? 3.0 : 2.0;
    const double nf = (double)px * p->ny * p->nz;
    if (nf * span * h->esize <= 4294967295.0) h->px = px;
  }
  // Plane stride: 256 bytes more than the plane (rounded to 256 bytes), so
  // that the 2Q planes a site's loads and stores touch do not all start at
  // one offset modulo a large power of two (256 x 128 x 128 channel: 16 MiB
  // planes; with the extra 256 bytes the FP32 read-once collision went from
  // 417 to 396 us, the FP16 total step from 17919 to 18709 MLUPS; 1 KiB and
  // 256 KiB extra gave nothing).  The moment scheme's 15 moment and 11
  // pre-collision moment planes take the same stride (its collision pass
  // 115 -> 103 us, the step 13326 -> 13876 MLUPS).
  {
    const char* env = std::getenv("LB_PLANE_PAD");  // measurement override: "0" keeps plain planes
    const bool plain = env && !std::strcmp(env, "0");
    const size_t g = 256 / h->esize;
    const size_t nf = (size_t)h->px * p->ny * p->nz;
    const size_t padded = (nf + g - 1) / g * g + g;
    const double span = p->lattice == LB_D2Q9 ? 3.0 : 2.0;
    h->NF = (!plain && (double)padded * span * h->esize <= 4294967295.0) ? padded : nf;
    // the same for the planes of N sites that the passes read and write
    // together (the four scalars, P of both colours)
    const size_t ns = (N + 63) / 64 * 64 + 64;
    h->NS = (h->moments() || plain) ? N : ns;
  }
  const size_t pop =
      h->moments() ? (size_t)LLB_NM * h->NF * h->esize : (h->total ? 1ull : 2ull) * h->q * h->NF * h->esize;
#define ALLOC(ptr, bytes)                                              \
  do {                                                                 \
    int r_ = dev_alloc((void**)&(ptr), (bytes), #ptr);                 \
    if (r_) { lb_destroy(h); return r_; }                              \
  } while (0)
  // in place: one copy of the populations, and one of the recolouring
  // scalars (the phase pass reads them, the collision pass rewrites them
  // afterwards; no pass does both)
  ALLOC(h->f[0], pop);
  if (!h->in_place()) ALLOC(h->f[1], pop);
  if (h->moments()) ALLOC(h->W, (size_t)LLB_NW * h->NF * h->esize);
  if (h->total) {
    ALLOC(h->sc[0], sizeof(float) * NSC * h->NS);
    if (!h->in_place()) ALLOC(h->sc[1], sizeof(float) * NSC * h->NS);
  }
  ALLOC(h->phi, N * h->rsize);
  if (h->ro) {
    ALLOC(h->phi2, N * h->rsize);
    ALLOC(h->ro_part, 2 * h->NS * h->rsize);
    // the read-once collision with FP32 arithmetic measured fastest with
    // about 2048 workgroups, half the march depth of the rule above (256 x
    // 128 x 128 channel: per-colour FP32 step 0.4616 -> 0.4478 ms, FP32 total
    // layout 0.3272 -> 0.3029 ms; FP64 was fastest at 16 planes)
    if (h->rsize == 4 && !std::getenv("LB_Z_PER_BLOCK")) {
      const long bxy = (long)((p->nx + TILE_X - 1) / TILE_X) * ((p->ny + TILE_Y - 1) / TILE_Y);
      long zb = (bxy * p->nz) / 2048;
      if (zb < 1) zb = 1;
      if (zb > 16) zb = 16;
      if (zb > p->nz) zb = p->nz;
      h->z_per_block = (int)zb;
    }
  }
  ALLOC(h->rho_a, N * h->rsize);
  ALLOC(h->rho_b, N * h->rsize);
  ALLOC(h->u, 3 * N * h->rsize);
  ALLOC(h->fnc, 3 * N * h->rsize);
  ALLOC(h->flags, N);
  ALLOC(h->labels, N * 4);
  ALLOC(h->diag_partial, sizeof(double) * DIAG_BLOCKS * DG_COUNT);
  ALLOC(h->diag_out, sizeof(double) * DG_COUNT);
  ALLOC(h->ccl_count, sizeof(unsigned int));
#undef ALLOC
  if (h->ro) {
    int rc = ro_plan(h);
    if (rc) { lb_destroy(h); return rc; }
  }
  *out = h;
  g_err.clear();
  return LB_OK;
}

// march depth of the read-once collision launch and the halo blocks it needs
// (scatter_geom.hpp); grows the halo buffer when the depth needs more
static int ro_plan(lb_handle* h) {
  const lb_params& p = h->p;
  // the handle's march depth as it is (the default is chosen for the
  // read-once pass at create).  The depth fixes which sums the combine pass
  // adds (tile-march edges), so both streaming modes take the same one and
  // give the same results bit for bit.
  long zb = h->z_per_block;
  if (zb > p.nz) zb = p.nz;
  h->ro_zb = (int)zb;
  HaloGeom g{};
  g.TX = TILE_X; g.TY = TILE_Y; g.zb = h->ro_zb;
  g.nx = p.nx; g.ny = p.ny; g.nz = p.nz;
  g.dims = h->d;
  g.tiles_x = (p.nx + TILE_X - 1) / TILE_X;
  g.tiles_y = (p.ny + TILE_Y - 1) / TILE_Y;
  g.marches = (p.nz + h->ro_zb - 1) / h->ro_zb;
  const size_t need = (size_t)g.entries() * 2 * h->rsize;
  if (need > h->ro_halo_bytes) {
    (void)hipSetDevice(h->device);
    if (h->ro_halo) {
      HIP_TRY(hipStreamSynchronize(h->stream));
      HIP_TRY(hipFree(h->ro_halo));
      h->ro_halo = nullptr;
      h->ro_halo_bytes = 0;
    }
    int rc = dev_alloc(&h->ro_halo, need, "scatter halo blocks");
    if (rc) return rc;
    h->ro_halo_bytes = need;
  }
  return LB_OK;
}

int lb_init_droplets(lb_handle* h, int channel, int n, const double* centres, const double* radii, double width,
                     double phi_in) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (h->ensemble()) {
    if (channel < 0 || channel >= (int)h->chans.size()) return fail(LB_EINVAL, "channel %d out of range", channel);
    int rc = lb_init_droplets(h->chans[channel], 0, n, centres, radii, width, phi_in);
    if (rc) return rc;
    h->t = 0;
    h->initialised = true;
    for (lb_handle* c : h->chans) h->initialised = h->initialised && c->initialised;
    return LB_OK;
  }
  if (channel != 0) return fail(LB_EINVAL, "channel %d out of range", channel);
  if (n < 0 || (n > 0 && (!centres || !radii))) return fail(LB_EINVAL, "bad droplet list");
  if (!(width > 0.0)) return fail(LB_EINVAL, "width must be positive");
  if (!(phi_in == 1.0 || phi_in == -1.0)) return fail(LB_EINVAL, "phi_in must be +1 or -1");
  std::vector<double> host(4 * (size_t)(n > 0 ? n : 1), 0.0);
  for (int d = 0; d < n; ++d) {
    for (int a = 0; a < 3; ++a) host[4 * d + a] = centres[3 * d + a];
    host[4 * d + 3] = radii[d];
    if (!(radii[d] >= 0.0) || !std::isfinite(centres[3 * d]) || !std::isfinite(centres[3 * d + 1]) ||
        !std::isfinite(centres[3 * d + 2]))
      return fail(LB_EINVAL, "droplet %d has a bad centre or radius", d);
  }
  (void)hipSetDevice(h->device);
  if (n > h->drops_cap) {
    if (h->drops) HIP_TRY(hipFree(h->drops));
    h->drops = nullptr;
    h->drops_cap = 0;
    int r = dev_alloc((void**)&h->drops, sizeof(double) * 4 * n, "drops");
    if (r) return r;
    h->drops_cap = n;
  }
  if (n > 0) HIP_TRY(hipMemcpyAsync(h->drops, host.data(), sizeof(double) * 4 * n, hipMemcpyHostToDevice, h->stream));
  InitArgs a{};
  a.nx = h->p.nx; a.ny = h->p.ny; a.nz = h->p.nz; a.dims = h->d;
  a.wall_x = h->p.wall[0]; a.wall_y = h->p.wall[1]; a.wall_z = h->p.wall[2];
  a.N = h->N; a.px = h->px; a.NF = (uint32_t)h->NF; a.NS = (uint32_t)h->NS; a.QN = (uint64_t)h->q * h->NF;
  a.ndrop = n;
  a.width = width; a.phi_in = phi_in; a.rho0 = h->p.rho0;
  a.u0x = h->p.u0[0]; a.u0y = h->p.u0[1]; a.u0z = h->d == 3 ? h->p.u0[2] : 0.0;
  a.half_rho0 = 0.5 * h->p.rho0;
  a.phi_I = h->p.phi_interface;
  // the state goes into the current copy, so an ensemble keeps one parity
  h->pcur = h->pfield = 0;
  h->phi_ready = false;
  if (h->moments())
    HIP_TRY(h->llb->init(h->p.storage, h->f[h->cur], h->phi, h->field_ptrs(), h->drops, a, h->stream));
  else
    HIP_TRY(h->ops->init(h->p.storage, h->f[h->cur], h->sc[h->cur], h->phi, h->field_ptrs(), h->drops, a, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));  // the host droplet list goes out of scope
  h->t = 0;
  h->ip_odd = 0;
  h->initialised = true;
  h->fields_valid = true;
  return LB_OK;
}

// record the first (begin) or second (end) event of pair slot `k`; grows the pool
static int prof_mark(lb_handle* h, int kind, bool begin) {
  if (!h->prof_on) return LB_OK;
  if (begin) {
    if (2 * (h->prof_used + 1) > h->prof_events.size()) {
      for (int j = 0; j < 2; ++j) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        h->prof_events.push_back(e);
      }
      h->prof_kind.push_back(kind);
    }
    h->prof_kind[h->prof_used] = kind;
    HIP_TRY(hipEventRecord(h->prof_events[2 * h->prof_used], h->stream));
  } else {
    HIP_TRY(hipEventRecord(h->prof_events[2 * h->prof_used + 1], h->stream));
    h->prof_used += 1;
  }
  return LB_OK;
}

static int run_diag(lb_handle* h) {
  DiagArgs a{};
  a.N = h->N;
  a.fx = h->p.body_force[0]; a.fy = h->p.body_force[1]; a.fz = h->d == 3 ? h->p.body_force[2] : 0.0;
  a.umax_ok = 0.3;
  if (h->p.storage == LB_F64) {
    k_diag_partial<double><<<DIAG_BLOCKS, DIAG_THREADS, 0, h->stream>>>(
        (const double*)h->rho_a, (const double*)h->rho_b, (const double*)h->u, (const double*)h->fnc,
        (const double*)h->phi_field(), h->diag_partial, a);
  } else {
    k_diag_partial<float><<<DIAG_BLOCKS, DIAG_THREADS, 0, h->stream>>>(
        (const float*)h->rho_a, (const float*)h->rho_b, (const float*)h->u, (const float*)h->fnc,
        (const float*)h->phi_field(), h->diag_partial, a);
  }
  HIP_TRY(hipGetLastError());
  k_diag_final<<<1, DIAG_THREADS, 0, h->stream>>>(h->diag_partial, DIAG_BLOCKS, h->diag_out);
  HIP_TRY(hipGetLastError());
  return LB_OK;
}

// ---------------------------------------------------------------- ensembles
// channel table and work lists for the current tuning
static int ensemble_plan(lb_handle* h) {
  const int nch = (int)h->chans.size();
  const int zb = h->tune.z_per_block;
  std::vector<ChannelDev> tab(nch);
  std::vector<uint32_t> tiles(nch);
  std::vector<uint32_t> nblocks(nch, 0);  // read-once: combine blocks per channel
  for (int c = 0; c < nch; ++c) {
    lb_handle* s = h->chans[c];
    s->z_per_block = zb;  // also the per-channel launches' tiling
    if (s->ro) {
      // halo blocks for this march depth (the stream is drained first if
      // they grow)
      int rc = ro_plan(s);
      if (rc) return rc;
    }
    ChannelDev& d = tab[c];
    std::memset(&d, 0, sizeof d);
    d.a = s->step_args();
    d.a.tiles_x = (s->p.nx + TILE_X - 1) / TILE_X;
    d.a.tiles_y = (s->p.ny + TILE_Y - 1) / TILE_Y;
    const uint32_t nzb = (uint32_t)((s->p.nz + zb - 1) / zb);
    d.ntiles = (uint32_t)d.a.tiles_x * d.a.tiles_y * nzb;
    if (d.ntiles > ITEM_TILE_MASK + 1) return fail(LB_EINVAL, "channel %d has too many tiles (%u)", c, d.ntiles);
    d.f[0] = s->f[0];
    d.f[1] = s->f[1];
    d.sc[0] = s->sc[0];
    d.sc[1] = s->sc[1];
    d.phi = s->phi;
    d.fo = s->field_ptrs();
    if (s->ro) {
      // the read-once launches use the march depth the halo blocks are sized for
      d.a.z_per_block = s->ro_zb;
      d.phis[0] = s->phi_at(0);
      d.phis[1] = s->phi_at(1);
      d.part = s->ro_part;
      d.halo = s->ro_halo;
      const uint32_t groups = (uint32_t)((s->ro_zb + COMBINE_PLANES - 1) / COMBINE_PLANES);
      nblocks[c] = (uint32_t)d.a.tiles_x * d.a.tiles_y * nzb * groups;
      if (nblocks[c] > ITEM_TILE_MASK + 1)
        return fail(LB_EINVAL, "channel %d has too many combine blocks (%u)", c, nblocks[c]);
    }
    tiles[c] = d.ntiles;
  }
  h->ens_cached = false;
  for (lb_handle* s : h->chans)
    if (((size_t)s->px * h->esize) % 64 != 0) h->ens_cached = true;
  if (const char* env = std::getenv("LB_ENSEMBLE_STORES")) {
    // measurement override: "nt" (non-temporal) or "cached"
    if (!std::strcmp(env, "nt")) h->ens_cached = false;
    else if (!std::strcmp(env, "cached")) h->ens_cached = true;
  }
  // largest channels first, so that the small ones fill the tail of a launch
  std::vector<int> order(nch);
  for (int c = 0; c < nch; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return tiles[a] > tiles[b]; });
  std::vector<uint32_t> ph, co, cb;
  for (int k = 0; k < nch; ++k) {
    const uint32_t c = (uint32_t)order[k];
    for (uint32_t t = 0; t < tiles[c]; ++t) {
      ph.push_back((c << ITEM_CH_SHIFT) | t);
      co.push_back(ITEM_COLLIDE | (c << ITEM_CH_SHIFT) | t);
    }
    for (uint32_t t = 0; t < nblocks[c]; ++t) cb.push_back((c << ITEM_CH_SHIFT) | t);
  }
  (void)hipSetDevice(h->device);
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (void** b : {(void**)&h->d_chans, (void**)&h->d_items_ph, (void**)&h->d_items_co, (void**)&h->d_items_cb})
    if (*b) {
      HIP_TRY(hipFree(*b));
      *b = nullptr;
    }
  if (h->graph) {
    HIP_TRY(hipGraphExecDestroy(h->graph));
    h->graph = nullptr;
  }
  int rc = 0;
  if ((rc = dev_alloc((void**)&h->d_chans, sizeof(ChannelDev) * nch, "channel table"))) return rc;
  if ((rc = dev_alloc((void**)&h->d_items_ph, sizeof(uint32_t) * ph.size(), "work list"))) return rc;
  if ((rc = dev_alloc((void**)&h->d_items_co, sizeof(uint32_t) * co.size(), "work list"))) return rc;
  HIP_TRY(hipMemcpy(h->d_chans, tab.data(), sizeof(ChannelDev) * nch, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_items_ph, ph.data(), sizeof(uint32_t) * ph.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_items_co, co.data(), sizeof(uint32_t) * co.size(), hipMemcpyHostToDevice));
  h->n_items_ph = (uint32_t)ph.size();
  h->n_items_co = (uint32_t)co.size();
  h->n_items_cb = (uint32_t)cb.size();
  if (!cb.empty()) {
    if ((rc = dev_alloc((void**)&h->d_items_cb, sizeof(uint32_t) * cb.size(), "work list"))) return rc;
    HIP_TRY(hipMemcpy(h->d_items_cb, cb.data(), sizeof(uint32_t) * cb.size(), hipMemcpyHostToDevice));
  }
  return LB_OK;
}

// read-once ensembles: a channel whose phase field is not ready (after an
// initialisation or a restore), or not in the buffer of its state's parity,
// scatters its stored state first (bit for bit what the collision pass that
// stored it would have scattered) and combines it into phi_at(cur), so that
// the phase field and the populations share one parity
static int ensemble_ro_boot(lb_handle* h) {
  for (lb_handle* c : h->chans) {
    if (c->phi_ready && c->pcur == c->cur) continue;
    StepArgs b = c->step_args();
    b.z_per_block = c->ro_zb;
    const ScatterOut so{c->ro_part, c->ro_halo};
    HIP_TRY(h->ops->boot(h->p.storage, c->f[c->cur], c->sc[c->cur], so, b, h->stream));
    HIP_TRY(h->ops->combine(h->p.storage, so, c->phi_at(c->cur), b, h->stream));
    c->pcur = c->cur;
    c->phi_ready = true;
  }
  return LB_OK;
}

// one step of channel c with the given parity (per-channel mode): the
// read-once collision and combine passes, or the phase and collision passes
static int channel_launch(lb_handle* h, lb_handle* c, bool fields, int parity, hipStream_t s) {
  const bool nc = h->p.nc_mode == LB_NC_EXPLICIT;
  const int st = h->p.storage;
  const StepArgs a = c->step_args();
  int rc = 0;
  if (c->ro) {
    StepArgs b = a;
    b.z_per_block = c->ro_zb;
    const ScatterOut so{c->ro_part, c->ro_halo};
    if ((rc = prof_mark(h, 1, true))) return rc;
    HIP_TRY(h->ops->collide(st, nc, fields, c->f[parity], c->f[1 - parity], c->sc[1 - parity], c->phi_at(parity),
                            c->field_ptrs(), b, &so, s));
    if ((rc = prof_mark(h, 1, false))) return rc;
    if ((rc = prof_mark(h, 2, true))) return rc;
    HIP_TRY(h->ops->combine(st, so, c->phi_at(1 - parity), b, s));
    return prof_mark(h, 2, false);
  }
  if ((rc = prof_mark(h, 0, true))) return rc;
  HIP_TRY(h->ops->phase(st, c->f[parity], c->sc[parity], c->phi, a, s));
  if ((rc = prof_mark(h, 0, false))) return rc;
  if ((rc = prof_mark(h, 1, true))) return rc;
  HIP_TRY(h->ops->collide(st, nc, fields, c->f[parity], c->f[1 - parity], c->sc[1 - parity], c->phi,
                          c->field_ptrs(), a, nullptr, s));
  return prof_mark(h, 1, false);
}

// enqueue one ensemble step with the given parity on stream s; while
// profiling (never under capture) the phase launches and the collision
// launches are timed separately
static int ensemble_launch(lb_handle* h, bool fields, int parity, hipStream_t s) {
  const bool nc = h->p.nc_mode == LB_NC_EXPLICIT;
  int rc = 0;
  if (h->tune.mode == LB_ENSEMBLE_BATCHED && h->ro) {
    // read-once: every channel's collision tile-marches (with the scatter),
    // then every channel's combine blocks
    if ((rc = prof_mark(h, 1, true))) return rc;
    HIP_TRY(h->ops->ensemble_ro(h->p.storage, nc, fields, false, h->ens_cached, h->d_chans, h->d_items_co,
                                h->n_items_co, parity, s));
    if ((rc = prof_mark(h, 1, false))) return rc;
    if ((rc = prof_mark(h, 2, true))) return rc;
    HIP_TRY(h->ops->ensemble_ro(h->p.storage, nc, fields, true, false, h->d_chans, h->d_items_cb, h->n_items_cb,
                                parity, s));
    return prof_mark(h, 2, false);
  }
  if (h->tune.mode == LB_ENSEMBLE_BATCHED) {
    if ((rc = prof_mark(h, 0, true))) return rc;
    HIP_TRY(h->ops->ensemble(h->p.storage, nc, fields, true, h->d_chans, h->d_items_ph, h->n_items_ph, parity, s));
    if ((rc = prof_mark(h, 0, false))) return rc;
    if ((rc = prof_mark(h, 1, true))) return rc;
    HIP_TRY(h->ops->ensemble(h->p.storage, nc, fields, false, h->d_chans, h->d_items_co, h->n_items_co, parity, s));
    return prof_mark(h, 1, false);
  }
  // channel after channel, each channel's passes back to back: the channel's
  // state (a few hundred MB) is then still in the MI355X's 256 MB last-level
  // cache in good part when the second pass reads it
  for (lb_handle* c : h->chans)
    if ((rc = channel_launch(h, c, fields, parity, s))) return rc;
  return LB_OK;
}

// capture two non-field steps (parity 0, then 1) into a graph
static int ensemble_graph(lb_handle* h) {
  if (h->graph) return LB_OK;
  hipStream_t cap = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  int rc = LB_OK;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = fail(LB_EHIP, "hipStreamBeginCapture failed");
  } else {
    const int r0 = ensemble_launch(h, false, 0, cap);
    const int r1 = r0 ? r0 : ensemble_launch(h, false, 1, cap);
    const hipError_t e = hipStreamEndCapture(cap, &g);
    if (r1) rc = r1;
    else if (e != hipSuccess || !g) rc = fail(LB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    else if (hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0) != hipSuccess)
      rc = fail(LB_EHIP, "hipGraphInstantiate failed");
  }
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cap);
  if (rc) h->graph = nullptr;
  return rc;
}

static void ensemble_advance(lb_handle* h, bool fields) {
  h->cur = 1 - h->cur;
  h->t += 1;
  for (lb_handle* c : h->chans) {
    if (c->ro) {
      // the step read phi_at(pcur) and its combine pass wrote the other one
      if (fields) c->pfield = c->pcur;
      c->pcur = 1 - c->pcur;
    }
    c->cur = h->cur;
    c->t += 1;
    if (fields) c->fields_valid = true;
  }
}

static int ensemble_step(lb_handle* h, int nsteps) {
  for (lb_handle* c : h->chans)
    if (!c->initialised) return fail(LB_EINVAL, "every channel must be initialised before stepping");
  if (h->ro && nsteps > 0) {
    int rc = ensemble_ro_boot(h);
    if (rc) return rc;
  }
  // per-channel mode without the watchdog: the channels are independent, so
  // each takes all nsteps before the next one starts.  A channel's state
  // (up to a few hundred MB) then stays largely in the 256 MB last-level
  // cache from one pass to the next.  The results are those of the
  // step-by-step order, bit for bit.
  if (h->tune.mode == LB_ENSEMBLE_PER_CHANNEL && h->p.diag_every <= 0 && nsteps > 1) {
    int rc = 0;
    for (lb_handle* c : h->chans)
      for (int k = 0; k < nsteps; ++k)
        if ((rc = channel_launch(h, c, k == nsteps - 1, (h->cur + k) & 1, h->stream))) return rc;
    for (int k = 0; k < nsteps; ++k) ensemble_advance(h, k == nsteps - 1);
    return LB_OK;
  }
  int s = 0;
  while (s < nsteps) {
    const bool diag_on = h->p.diag_every > 0;
    const bool diag_now = diag_on && ((h->t + 1) % h->p.diag_every) == 0;
    const bool fields = (s == nsteps - 1) || diag_now;
    // two non-field steps from the captured graph when the parity lines up
    if (!fields && !diag_on && h->tune.use_graph && h->cur == 0 && s + 2 <= nsteps - 1 && !h->prof_on) {
      int rc = ensemble_graph(h);
      if (rc) return rc;
      HIP_TRY(hipGraphLaunch(h->graph, h->stream));
      ensemble_advance(h, false);
      ensemble_advance(h, false);
      s += 2;
      continue;
    }
    int rc = ensemble_launch(h, fields, h->cur, h->stream);
    if (rc) return rc;
    ensemble_advance(h, fields);
    s += 1;
    if (diag_now) {
      for (size_t c = 0; c < h->chans.size(); ++c) {
        lb_handle* ch = h->chans[c];
        if ((rc = run_diag(ch))) return rc;
        double bad = 0.0;
        HIP_TRY(hipMemcpyAsync(&bad, ch->diag_out + DG_BAD, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        if (bad > 0.0)
          return fail(LB_ENUMERIC, "watchdog at step %lld, channel %zu: %.0f bad sites", h->t, c, bad);
      }
    }
  }
  return LB_OK;
}

// Enqueue one single-lattice step on stream s.  It reads the handle's state
// (buffer parities, in-place kind, whether the read-once phase field is
// ready) and changes none of it: single_advance does that.  Profiling marks
// go to the handle's stream while profiling is on, which excludes graph
// capture (then s is the handle's stream).
static int single_launch(lb_handle* h, bool fields, hipStream_t s) {
  StepArgs a = h->step_args();
  a.step = (uint32_t)h->t;  // keys the stochastic rounding of this step's stores
  const FieldPtrs fo = h->field_ptrs();
  const bool nc = h->p.nc_mode == LB_NC_EXPLICIT;
  const bool mlp = h->p.nc_mode == LB_NC_MLP;
  const int st = h->p.storage;
  int r = prof_mark(h, 0, true);
  if (r) return r;
  if (h->moments()) {
    // pass 1 rebuilds the pulled populations from the upstream moments,
    // pass 2 writes the new moments into the other copy
    HIP_TRY(h->llb->pull(st, h->f[h->cur], h->W, h->phi, a, s));
    if ((r = prof_mark(h, 0, false))) return r;
    if ((r = prof_mark(h, 1, true))) return r;
    HIP_TRY(h->llb->collide(st, nc, fields, h->W, h->f[1 - h->cur], h->phi, fo, a, s));
    return prof_mark(h, 1, false);
  }
  if (h->ro) {
    // read-once step: the collision pass reads phi_at(pcur) and scatters
    // the next step's colour densities; the combine pass turns them into
    // the next phase field in the other buffer.  The first step after
    // lb_init_droplets / lb_set_state scatters the stored state first (the
    // bootstrap pass, bit for bit what the collision pass that stored it
    // would have scattered), so restarts repeat uninterrupted runs exactly.
    StepArgs b = a;
    b.z_per_block = h->ro_zb;
    const ScatterOut so{h->ro_part, h->ro_halo};
    void* phin = h->phi_at(h->pcur);
    void* phout = h->phi_at(1 - h->pcur);
    if (h->in_place()) {
      void* f = h->f[0];
      float* sc = h->sc[0];
      const int odd = h->ip_odd;
      if (!h->phi_ready) {
        // an initialised or restored state is canonical (odd == 0); the
        // phase pass covers any other case
        if (odd) {
          HIP_TRY(h->ip->phase_odd(st, f, sc, phin, a, s));
        } else {
          HIP_TRY(h->ops->boot(st, f, sc, so, b, s));
          HIP_TRY(h->ops->combine(st, so, phin, b, s));
        }
        if ((r = prof_mark(h, 0, false))) return r;
      }
      // (without the phase pass, the next mark reuses the open one)
      if ((r = prof_mark(h, 1, true))) return r;
      if (mlp) HIP_TRY(h->ip->collide_mlp(st, odd, fields, f, sc, phin, fo, b, h->mlp_net, &so, s));
      else HIP_TRY(h->ip->collide(st, odd, nc, fields, f, sc, phin, fo, b, &so, s));
    } else {
      void* fin = h->f[h->cur];
      void* fout = h->f[1 - h->cur];
      if (!h->phi_ready) {
        HIP_TRY(h->ops->boot(st, fin, h->sc[h->cur], so, b, s));
        HIP_TRY(h->ops->combine(st, so, phin, b, s));
        if ((r = prof_mark(h, 0, false))) return r;
      }
      if ((r = prof_mark(h, 1, true))) return r;
      if (mlp)
        HIP_TRY(h->ops->collide_mlp(st, fields, fin, fout, h->sc[1 - h->cur], phin, fo, b, h->mlp_net, &so, s));
      else
        HIP_TRY(h->ops->collide(st, nc, fields, fin, fout, h->sc[1 - h->cur], phin, fo, b, &so, s));
    }
    if ((r = prof_mark(h, 1, false))) return r;
    if ((r = prof_mark(h, 2, true))) return r;
    HIP_TRY(h->ops->combine(st, so, phout, b, s));
    return prof_mark(h, 2, false);
  }
  if (h->in_place()) {
    // one copy: even steps pull and push, odd steps work on the site's own slots
    void* f = h->f[0];
    float* sc = h->sc[0];
    const int odd = h->ip_odd;
    if (odd) HIP_TRY(h->ip->phase_odd(st, f, sc, h->phi, a, s));
    else HIP_TRY(h->ops->phase(st, f, sc, h->phi, a, s));
    if ((r = prof_mark(h, 0, false))) return r;
    if ((r = prof_mark(h, 1, true))) return r;
    if (mlp) HIP_TRY(h->ip->collide_mlp(st, odd, fields, f, sc, h->phi, fo, a, h->mlp_net, nullptr, s));
    else HIP_TRY(h->ip->collide(st, odd, nc, fields, f, sc, h->phi, fo, a, nullptr, s));
    return prof_mark(h, 1, false);
  }
  void* fin = h->f[h->cur];
  void* fout = h->f[1 - h->cur];
  HIP_TRY(h->ops->phase(st, fin, h->sc[h->cur], h->phi, a, s));
  if ((r = prof_mark(h, 0, false))) return r;
  if ((r = prof_mark(h, 1, true))) return r;
  if (mlp)
    HIP_TRY(h->ops->collide_mlp(st, fields, fin, fout, h->sc[1 - h->cur], h->phi, fo, a, h->mlp_net, nullptr, s));
  else
    HIP_TRY(h->ops->collide(st, nc, fields, fin, fout, h->sc[1 - h->cur], h->phi, fo, a, nullptr, s));
  return prof_mark(h, 1, false);
}

// the state change of one single-lattice step
static void single_advance(lb_handle* h, bool fields) {
  if (h->in_place() && !h->moments()) h->ip_odd = 1 - h->ip_odd;
  else h->cur = 1 - h->cur;
  if (h->ro) {
    if (fields) h->pfield = h->pcur;
    h->pcur = 1 - h->pcur;
    h->phi_ready = true;
  }
  h->t += 1;
  if (fields) h->fields_valid = true;
}

// the buffer parities a single-lattice graph was captured at; two steps
// bring them back
static int single_graph_key(const lb_handle* h) { return h->cur | (h->pcur << 1) | (h->ip_odd << 2); }

// capture two non-field single-lattice steps into a graph, starting at the
// current buffer parities (the read-once phase field must be ready)
static int single_graph(lb_handle* h) {
  if (h->graph) return LB_OK;
  hipStream_t cap = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  int rc = LB_OK;
  // the launches read the handle's state: step it through the two steps
  // while capturing and put it back afterwards
  const int cur0 = h->cur, pcur0 = h->pcur, pfield0 = h->pfield, odd0 = h->ip_odd;
  const bool ready0 = h->phi_ready, valid0 = h->fields_valid;
  const long long t0 = h->t;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = fail(LB_EHIP, "hipStreamBeginCapture failed");
  } else {
    int r = single_launch(h, false, cap);
    if (!r) {
      single_advance(h, false);
      r = single_launch(h, false, cap);
    }
    const hipError_t e = hipStreamEndCapture(cap, &g);
    if (r) rc = r;
    else if (e != hipSuccess || !g) rc = fail(LB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    else if (hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0) != hipSuccess)
      rc = fail(LB_EHIP, "hipGraphInstantiate failed");
  }
  h->cur = cur0;
  h->pcur = pcur0;
  h->pfield = pfield0;
  h->ip_odd = odd0;
  h->phi_ready = ready0;
  h->t = t0;
  h->fields_valid = valid0;
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cap);
  if (rc) h->graph = nullptr;
  else h->graph_key = single_graph_key(h);
  return rc;
}

static int single_graph_drop(lb_handle* h) {
  if (!h->graph) return LB_OK;
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipGraphExecDestroy(h->graph));
  h->graph = nullptr;
  return LB_OK;
}

int lb_step(lb_handle* h, int nsteps) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  if (h->ensemble()) {
    (void)hipSetDevice(h->device);
    return ensemble_step(h, nsteps);
  }
  if (!h->initialised) return fail(LB_EINVAL, "call lb_init_droplets or lb_set_state first");
  if (h->p.nc_mode == LB_NC_MLP && !h->mlp_weights)
    return fail(LB_EINVAL, "LB_NC_MLP needs network parameters (lb_mlp_set_weights or lb_mlp_train)");
  (void)hipSetDevice(h->device);
  // graph replays: pairs of non-field steps at the captured parities, without
  // the watchdog, profiling or stochastic rounding (whose key is the step)
  const bool graph_ok = h->tune.use_graph && h->p.diag_every <= 0 && h->p.rounding != LB_ROUND_STOCHASTIC;
  int s = 0;
  while (s < nsteps) {
    const bool diag_now = h->p.diag_every > 0 && ((h->t + 1) % h->p.diag_every) == 0;
    const bool fields = (s == nsteps - 1) || diag_now;
    if (graph_ok && !fields && s + 2 <= nsteps - 1 && !h->prof_on && (!h->ro || h->phi_ready)) {
      // a graph of neither this parity nor the next (after a restart that
      // left the buffers paired differently) is captured again
      const int key = single_graph_key(h);
      const int flip = ((h->in_place() && !h->moments()) ? 4 : 1) | (h->ro ? 2 : 0);
      if (h->graph && h->graph_key != key && h->graph_key != (key ^ flip)) {
        int r = single_graph_drop(h);
        if (r) return r;
      }
      int r = single_graph(h);
      if (r) return r;
      if (h->graph_key == key) {
        HIP_TRY(hipGraphLaunch(h->graph, h->stream));
        single_advance(h, false);
        single_advance(h, false);
        s += 2;
        continue;
      }
      // the other parity: one step directly brings it in line
    }
    int r = single_launch(h, fields, h->stream);
    if (r) return r;
    single_advance(h, fields);
    s += 1;
    if (diag_now) {
      r = run_diag(h);
      if (r) return r;
      double bad = 0.0;
      HIP_TRY(hipMemcpyAsync(&bad, h->diag_out + DG_BAD, sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
      if (bad > 0.0)
        return fail(LB_ENUMERIC, "watchdog at step %lld: %.0f sites with NaN/Inf, rho <= 0 or |u| > 0.3", h->t, bad);
    }
  }
  return LB_OK;
}

static int run_labels(lb_handle* h, unsigned int* count_host) {
  CclArgs c{};
  c.nx = h->p.nx; c.ny = h->p.ny; c.nz = h->p.nz; c.dims = h->d;
  c.wall_x = h->p.wall[0]; c.wall_y = h->p.wall[1]; c.wall_z = h->p.wall[2];
  c.N = h->N;
  const dim3 grid((h->N + 255) / 256), block(256);
  if (h->p.storage == LB_F64)
    k_ccl_init<double><<<grid, block, 0, h->stream>>>((const double*)h->phi_field(), h->labels, h->N);
  else
    k_ccl_init<float><<<grid, block, 0, h->stream>>>((const float*)h->phi_field(), h->labels, h->N);
  HIP_TRY(hipGetLastError());
  k_ccl_merge<<<grid, block, 0, h->stream>>>(h->labels, c);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemsetAsync(h->ccl_count, 0, sizeof(unsigned int), h->stream));
  k_ccl_flatten<<<grid, block, 0, h->stream>>>(h->labels, h->N, h->ccl_count);
  HIP_TRY(hipGetLastError());
  if (count_host) {
    HIP_TRY(hipMemcpyAsync(count_host, h->ccl_count, sizeof(unsigned int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  return LB_OK;
}

int lb_fields(lb_handle* h, int channel, unsigned mask, void* const* dst, int dst_on_device) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (h->ensemble()) {
    if (channel < 0 || channel >= (int)h->chans.size()) return fail(LB_EINVAL, "channel %d out of range", channel);
    return lb_fields(h->chans[channel], 0, mask, dst, dst_on_device);
  }
  if (channel != 0) return fail(LB_EINVAL, "channel %d out of range", channel);
  if (mask >> LB_NUM_FIELDS) return fail(LB_EINVAL, "unknown field bits in mask 0x%x", mask);
  if (mask && !dst) return fail(LB_EINVAL, "dst is NULL");
  if (!h->fields_valid) return fail(LB_EINVAL, "no fields yet: initialise or take a step after lb_set_state");
  for (int b = 0; b < LB_NUM_FIELDS; ++b)
    if ((mask >> b) & 1u)
      if (!dst[b]) return fail(LB_EINVAL, "dst[%d] is NULL for a selected field", b);
  (void)hipSetDevice(h->device);
  const size_t N = h->N, r = h->rsize;
  const void* src[LB_NUM_FIELDS] = {h->rho_a, h->rho_b, h->phi_field(), h->u, h->fnc, h->flags, h->labels};
  const size_t bytes[LB_NUM_FIELDS] = {N * r, N * r, N * r, 3 * N * r, 3 * N * r, N, 4 * N};
  if (mask & LB_FIELD_LABELS) {
    int rc = run_labels(h, nullptr);
    if (rc) return rc;
  }
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  for (int b = 0; b < LB_NUM_FIELDS; ++b)
    if ((mask >> b) & 1u) HIP_TRY(hipMemcpyAsync(dst[b], src[b], bytes[b], kind, h->stream));
  if (!dst_on_device) HIP_TRY(hipStreamSynchronize(h->stream));
  return LB_OK;
}

int lb_diagnostics(lb_handle* h, int channel, double out[8]) {
  if (!h || !out) return fail(LB_EINVAL, "NULL argument");
  if (h->ensemble()) {
    if (channel < 0 || channel >= (int)h->chans.size()) return fail(LB_EINVAL, "channel %d out of range", channel);
    return lb_diagnostics(h->chans[channel], 0, out);
  }
  if (channel != 0) return fail(LB_EINVAL, "channel %d out of range", channel);
  if (!h->fields_valid) return fail(LB_EINVAL, "no fields yet: initialise or take a step after lb_set_state");
  (void)hipSetDevice(h->device);
  int rc = run_diag(h);
  if (rc) return rc;
  double d[DG_COUNT];
  HIP_TRY(hipMemcpyAsync(d, h->diag_out, sizeof d, hipMemcpyDeviceToHost, h->stream));
  unsigned int count = 0;
  rc = run_labels(h, &count);  // synchronises
  if (rc) return rc;
  out[0] = d[DG_RHOA];
  out[1] = d[DG_RHOB];
  out[2] = d[DG_JX];
  out[3] = d[DG_JY];
  out[4] = d[DG_JZ];
  out[5] = d[DG_UMAX];
  out[6] = (double)count;
  out[7] = (d[DG_N_IN] > 0 && d[DG_N_OUT] > 0)
               ? (d[DG_RHO_IN] / d[DG_N_IN] - d[DG_RHO_OUT] / d[DG_N_OUT]) / 3.0
               : std::nan("");
  return LB_OK;
}

// The populations in the canonical layout after an odd number of in-place
// steps: gathered by colour block straight into a device destination, or
// plane by plane through a one-plane staging buffer for a host destination.
static int canonical_state(lb_handle* h, void* dst, int dst_on_device) {
  const StepArgs a = h->step_args();
  const int nblk = h->total ? 1 : 2;
  const size_t plane = (size_t)h->N * h->esize;     // canonical plane
  const size_t fplane = h->NF * h->esize;            // device plane (padded stride)
  if (dst_on_device) {
    for (int k = 0; k < nblk; ++k)
      HIP_TRY(h->ip->canonical(h->p.storage, (const char*)h->f[0] + k * h->q * fplane, (char*)dst + k * h->q * plane,
                               0, h->q, a, h->stream));
    return LB_OK;
  }
  void* tmp = nullptr;
  int rc = dev_alloc(&tmp, plane, "canonical staging plane");
  if (rc) return rc;
  hipError_t e = hipSuccess;
  for (int k = 0; k < nblk && e == hipSuccess; ++k)
    for (int i = 0; i < h->q && e == hipSuccess; ++i) {
      e = h->ip->canonical(h->p.storage, (const char*)h->f[0] + k * h->q * fplane, tmp, i, i + 1, a, h->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync((char*)dst + (k * h->q + i) * plane, tmp, plane, hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
  (void)hipStreamSynchronize(h->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(LB_EHIP, "canonical state: %s", hipGetErrorString(e));
  return LB_OK;
}

static size_t state_size(const lb_handle* h, size_t* pop_bytes) {
  if (h->ensemble()) {
    size_t tot = 0;
    for (const lb_handle* c : h->chans) tot += state_size(c, nullptr);
    if (pop_bytes) *pop_bytes = 0;
    return tot;
  }
  const size_t pop = h->moments() ? (size_t)LLB_NM * h->N * h->esize
                                   : (h->total ? 1ull : 2ull) * h->q * h->N * h->esize;
  if (pop_bytes) *pop_bytes = pop;
  return pop + (h->total ? sizeof(float) * NSC * h->N : 0);
}

int lb_state_bytes(const lb_handle* h, size_t* bytes) {
  if (!h || !bytes) return fail(LB_EINVAL, "NULL argument");
  *bytes = state_size(h, nullptr);
  return LB_OK;
}

int lb_get_state(lb_handle* h, void* dst, size_t bytes, int dst_on_device) {
  if (!h || !dst) return fail(LB_EINVAL, "NULL argument");
  size_t pop = 0;
  const size_t need = state_size(h, &pop);
  if (bytes != need) return fail(LB_EINVAL, "state is %zu bytes, got %zu", need, bytes);
  (void)hipSetDevice(h->device);
  if (h->ensemble()) {
    size_t off = 0;
    for (lb_handle* c : h->chans) {
      const size_t b = state_size(c, nullptr);
      int rc = lb_get_state(c, (char*)dst + off, b, dst_on_device);
      if (rc) return rc;
      off += b;
    }
    return LB_OK;
  }
  const hipMemcpyKind k = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (h->in_place() && h->ip_odd) {
    int rc = canonical_state(h, dst, dst_on_device);
    if (rc) return rc;
  } else if (h->NF == h->N) {
    HIP_TRY(hipMemcpyAsync(dst, h->f[h->cur], pop, k, h->stream));
  } else {
    // padded rows and planes: the canonical state holds nx sites per row
    // and N per plane
    const size_t row = (size_t)h->p.nx * h->esize, plane = (size_t)h->N * h->esize;
    for (size_t i = 0; i < pop / plane; ++i)
      HIP_TRY(hipMemcpy2DAsync((char*)dst + i * plane, row, (const char*)h->f[h->cur] + i * h->NF * h->esize,
                               (size_t)h->px * h->esize, row, plane / row, k, h->stream));
  }
  if (h->total)
    HIP_TRY(hipMemcpy2DAsync((char*)dst + pop, sizeof(float) * h->N, h->sc[h->cur], sizeof(float) * h->NS,
                             sizeof(float) * h->N, NSC, k, h->stream));
  if (!dst_on_device) HIP_TRY(hipStreamSynchronize(h->stream));
  return LB_OK;
}

int lb_set_state(lb_handle* h, const void* src, size_t bytes, int src_on_device) {
  if (!h || !src) return fail(LB_EINVAL, "NULL argument");
  size_t pop = 0;
  const size_t need = state_size(h, &pop);
  if (bytes != need) return fail(LB_EINVAL, "state is %zu bytes, got %zu", need, bytes);
  (void)hipSetDevice(h->device);
  if (h->ensemble()) {
    size_t off = 0;
    for (lb_handle* c : h->chans) {
      const size_t b = state_size(c, nullptr);
      int rc = lb_set_state(c, (const char*)src + off, b, src_on_device);
      if (rc) return rc;
      off += b;
    }
    h->initialised = true;
    return LB_OK;
  }
  const hipMemcpyKind k = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (h->NF == h->N) {
    HIP_TRY(hipMemcpyAsync(h->f[h->cur], src, pop, k, h->stream));
  } else {
    const size_t row = (size_t)h->p.nx * h->esize, plane = (size_t)h->N * h->esize;
    for (size_t i = 0; i < pop / plane; ++i)
      HIP_TRY(hipMemcpy2DAsync((char*)h->f[h->cur] + i * h->NF * h->esize, (size_t)h->px * h->esize,
                               (const char*)src + i * plane, row, row, plane / row, k, h->stream));
  }
  if (h->total)
    HIP_TRY(hipMemcpy2DAsync(h->sc[h->cur], sizeof(float) * h->NS, (const char*)src + pop, sizeof(float) * h->N,
                             sizeof(float) * h->N, NSC, k, h->stream));
  if (!src_on_device) HIP_TRY(hipStreamSynchronize(h->stream));
  h->ip_odd = 0;  // the state given is canonical
  h->initialised = true;
  h->fields_valid = false;
  h->phi_ready = false;
  return LB_OK;
}

int lb_step_count(const lb_handle* h, long long* t) {
  if (!h || !t) return fail(LB_EINVAL, "NULL argument");
  *t = h->t;
  return LB_OK;
}

int lb_profile_begin(lb_handle* h) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  h->prof_on = true;
  h->prof_used = 0;
  return LB_OK;
}

int lb_profile_end(lb_handle* h, double* ms_phase, double* ms_collide, double* ms_combine, int* n_phase,
                   int* n_collide, int* n_combine) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  (void)hipSetDevice(h->device);
  HIP_TRY(hipStreamSynchronize(h->stream));
  double t[3] = {0.0, 0.0, 0.0};
  int n[3] = {0, 0, 0};
  for (size_t k = 0; k < h->prof_used; ++k) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, h->prof_events[2 * k], h->prof_events[2 * k + 1]));
    t[h->prof_kind[k]] += ms;
    n[h->prof_kind[k]] += 1;
  }
  h->prof_on = false;
  h->prof_used = 0;
  if (ms_phase) *ms_phase = t[0];
  if (ms_collide) *ms_collide = t[1];
  if (ms_combine) *ms_combine = t[2];
  if (n_phase) *n_phase = n[0];
  if (n_collide) *n_collide = n[1];
  if (n_combine) *n_combine = n[2];
  return LB_OK;
}

int lb_sync(lb_handle* h) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  (void)hipSetDevice(h->device);
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LB_OK;
}

int lb_channel_count(const lb_handle* h, int* n) {
  if (!h || !n) return fail(LB_EINVAL, "NULL argument");
  *n = h->ensemble() ? (int)h->chans.size() : 1;
  return LB_OK;
}

int lb_get_tuning(const lb_handle* h, lb_tuning* t) {
  if (!h || !t) return fail(LB_EINVAL, "NULL argument");
  if (h->ensemble()) {
    *t = h->tune;
  } else {
    std::memset(t, 0, sizeof *t);
    t->z_per_block = h->z_per_block;
    t->use_graph = h->tune.use_graph;
  }
  return LB_OK;
}

int lb_set_tuning(lb_handle* h, const lb_tuning* t) {
  if (!h || !t) return fail(LB_EINVAL, "NULL argument");
  if (t->z_per_block < 1 || t->z_per_block > 4096) return fail(LB_EINVAL, "z_per_block must lie in [1, 4096]");
  if (t->use_graph != 0 && t->use_graph != 1) return fail(LB_EINVAL, "use_graph must be 0 or 1");
  if (!h->ensemble()) {
    // the graph holds the launch shapes and the read-once halo buffers
    (void)hipSetDevice(h->device);
    int rc = single_graph_drop(h);
    if (rc) return rc;
    h->z_per_block = t->z_per_block;
    h->tune.use_graph = t->use_graph;
    return h->ro ? ro_plan(h) : LB_OK;
  }
  if (t->mode != LB_ENSEMBLE_BATCHED && t->mode != LB_ENSEMBLE_PER_CHANNEL) return fail(LB_EINVAL, "unknown mode");
  const int zb_old = h->tune.z_per_block;
  h->tune = *t;
  h->tune.ms_per_step = 0.0;
  (void)hipSetDevice(h->device);
  if (zb_old != t->z_per_block || !h->d_items_ph) return ensemble_plan(h);
  if (h->graph) {
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipGraphExecDestroy(h->graph));
    h->graph = nullptr;
  }
  return LB_OK;
}

int lb_autotune(lb_handle* h, int steps, lb_tuning* best, double* results, int cap, int* n_results) {
  if (!h || !best) return fail(LB_EINVAL, "NULL argument");
  if (steps < 1) return fail(LB_EINVAL, "steps must be >= 1");
  if (!h->initialised && !h->ensemble()) return fail(LB_EINVAL, "initialise the state first");
  (void)hipSetDevice(h->device);
  std::vector<lb_tuning> cand;
  if (h->ensemble()) {
    // the per-channel mode launches each channel's passes directly (its
    // step count varies per call), so only the batched mode has graph
    // candidates
    for (int mode : {LB_ENSEMBLE_BATCHED, LB_ENSEMBLE_PER_CHANNEL})
      for (int zb : {1, 2, 4, 8, 16, 32})
        for (int graph : {0, 1}) {
          if (mode == LB_ENSEMBLE_PER_CHANNEL && graph) continue;
          lb_tuning t{};
          t.mode = mode;
          t.z_per_block = zb;
          t.use_graph = graph;
          cand.push_back(t);
        }
  } else {
    for (int zb : {1, 2, 4, 8, 16, 32})
      for (int graph : {0, 1})
        if (zb <= h->p.nz) {
          lb_tuning t{};
          t.z_per_block = zb;
          t.use_graph = graph;
          cand.push_back(t);
        }
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best_k = -1;
  double best_ms = 1e300;
  int rc = LB_OK;
  for (size_t k = 0; k < cand.size() && !rc; ++k) {
    if ((rc = lb_set_tuning(h, &cand[k]))) break;
    if ((rc = lb_step(h, 2))) break;  // warm-up (and graph capture)
    if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = fail(LB_EHIP, "hipEventRecord"); break; }
    if ((rc = lb_step(h, steps))) break;
    if (hipEventRecord(e1, h->stream) != hipSuccess) { rc = fail(LB_EHIP, "hipEventRecord"); break; }
    if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(LB_EHIP, "hipEventSynchronize"); break; }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double per = ms / steps;
    cand[k].ms_per_step = per;
    if (results && (int)k < cap) {
      results[4 * k + 0] = cand[k].mode;
      results[4 * k + 1] = cand[k].z_per_block;
      results[4 * k + 2] = cand[k].use_graph;
      results[4 * k + 3] = per;
    }
    if (per < best_ms) {
      best_ms = per;
      best_k = (int)k;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (n_results) *n_results = (int)cand.size();
  if (rc) return rc;
  if (best_k < 0) return fail(LB_EHIP, "no candidate ran");
  rc = lb_set_tuning(h, &cand[best_k]);
  if (rc) return rc;
  *best = cand[best_k];
  if (h->ensemble()) h->tune.ms_per_step = best_ms;
  return LB_OK;
}

// ------------------------------------------------------ learned closure
static int mlp_alloc(lb_handle* h) {
  if (h->mlp_theta) return LB_OK;
  int rc = 0;
  if ((rc = dev_alloc((void**)&h->mlp_theta, sizeof(float) * MLP_PARAMS, "closure parameters"))) return rc;
  if ((rc = dev_alloc((void**)&h->mlp_m1, sizeof(float) * MLP_PARAMS, "Adam moments"))) return rc;
  if ((rc = dev_alloc((void**)&h->mlp_m2, sizeof(float) * MLP_PARAMS, "Adam moments"))) return rc;
  // gradient plus one float for a batch loss nobody asked for
  if ((rc = dev_alloc((void**)&h->mlp_grad, sizeof(float) * (MLP_PARAMS + 1), "closure gradient"))) return rc;
  if ((rc = dev_alloc((void**)&h->mlp_lo, sizeof(float) * 64, "closure ranges"))) return rc;
  if ((rc = dev_alloc((void**)&h->mlp_bad, sizeof(uint32_t), "closure flag"))) return rc;
  if ((rc = dev_alloc((void**)&h->mlp_net, sizeof(MlpPacked), "packed closure"))) return rc;
  // empty ranges until set: every interface site takes the explicit scan
  float r[64];
  for (int k = 0; k < 32; ++k) {
    r[k] = INFINITY;
    r[32 + k] = -INFINITY;
  }
  HIP_TRY(hipMemcpy(h->mlp_lo, r, sizeof r, hipMemcpyHostToDevice));
  h->mlp_gmin = INFINITY;
  return LB_OK;
}

static int mlp_parts(lb_handle* h, int nparts) {
  if (nparts <= h->mlp_part_cap) return LB_OK;
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (h->mlp_part) HIP_TRY(hipFree(h->mlp_part));
  if (h->mlp_part_l) HIP_TRY(hipFree(h->mlp_part_l));
  h->mlp_part = nullptr;
  h->mlp_part_l = nullptr;
  h->mlp_part_cap = 0;
  int rc = 0;
  if ((rc = dev_alloc((void**)&h->mlp_part, sizeof(float) * MLP_PARAMS * (size_t)nparts, "partial gradients")))
    return rc;
  if ((rc = dev_alloc((void**)&h->mlp_part_l, sizeof(float) * (size_t)nparts, "partial losses"))) return rc;
  h->mlp_part_cap = nparts;
  return LB_OK;
}

static int mlp_pack(lb_handle* h) {
  k_mlp_pack<<<1, 256, 0, h->stream>>>(h->mlp_theta, h->mlp_lo, h->mlp_lo + 32, h->mlp_gmin, h->mlp_net);
  HIP_TRY(hipGetLastError());
  return LB_OK;
}

int lb_mlp_set_weights(lb_handle* h, const float* theta, long long n) {
  if (!h || !theta) return fail(LB_EINVAL, "NULL argument");
  if (n != MLP_PARAMS) return fail(LB_EINVAL, "expected %d parameters, got %lld", MLP_PARAMS, n);
  if (h->ensemble()) return fail(LB_EINVAL, "the learned closure is not available for ensembles");
  (void)hipSetDevice(h->device);
  int rc = mlp_alloc(h);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(h->mlp_theta, theta, sizeof(float) * MLP_PARAMS, hipMemcpyHostToDevice, h->stream));
  if ((rc = mlp_pack(h))) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->mlp_weights = true;
  return LB_OK;
}

int lb_mlp_get_weights(lb_handle* h, float* theta, long long n) {
  if (!h || !theta) return fail(LB_EINVAL, "NULL argument");
  if (n != MLP_PARAMS) return fail(LB_EINVAL, "expected %d parameters, got %lld", MLP_PARAMS, n);
  if (!h->mlp_weights) return fail(LB_EINVAL, "no network parameters set");
  (void)hipSetDevice(h->device);
  HIP_TRY(hipMemcpyAsync(theta, h->mlp_theta, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LB_OK;
}

int lb_mlp_set_ranges(lb_handle* h, const float* lo, const float* hi, float gmin) {
  if (!h || !lo || !hi) return fail(LB_EINVAL, "NULL argument");
  if (h->ensemble()) return fail(LB_EINVAL, "the learned closure is not available for ensembles");
  (void)hipSetDevice(h->device);
  int rc = mlp_alloc(h);
  if (rc) return rc;
  float r[64];
  for (int k = 0; k < 32; ++k) {
    r[k] = k < MLP_IN ? lo[k] : INFINITY;
    r[32 + k] = k < MLP_IN ? hi[k] : -INFINITY;
  }
  HIP_TRY(hipMemcpyAsync(h->mlp_lo, r, sizeof r, hipMemcpyHostToDevice, h->stream));
  h->mlp_gmin = gmin;
  if ((rc = mlp_pack(h))) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LB_OK;
}

int lb_mlp_get_ranges(lb_handle* h, float* lo, float* hi, float* gmin) {
  if (!h || !lo || !hi || !gmin) return fail(LB_EINVAL, "NULL argument");
  (void)hipSetDevice(h->device);
  int rc = mlp_alloc(h);
  if (rc) return rc;
  float r[64];
  HIP_TRY(hipMemcpyAsync(r, h->mlp_lo, sizeof r, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int k = 0; k < MLP_IN; ++k) {
    lo[k] = r[k];
    hi[k] = r[32 + k];
  }
  *gmin = h->mlp_gmin;
  return LB_OK;
}

// forward/backward over nb rows (idx == NULL: rows 0 .. nb-1), summed into
// mlp_grad, loss into loss_dst
static int mlp_fwdbwd(lb_handle* h, const float* rows, const float* targets, long long m, const int* idx, int nb,
                      float* loss_dst) {
  const int nparts = (nb + MLP_SB - 1) / MLP_SB;
  int rc = mlp_parts(h, nparts);
  if (rc) return rc;
  k_mlp_fwdbwd<<<nparts, MLP_TB, 0, h->stream>>>(
      h->mlp_theta, rows, targets, (const int32_t*)idx, nb, m, (float)(2.0 / (3.0 * nb)), h->mlp_part,
      h->mlp_part_l, h->mlp_bad);
  HIP_TRY(hipGetLastError());
  k_mlp_reduce<<<(MLP_PARAMS + 255) / 256, 256, 0, h->stream>>>(h->mlp_part, h->mlp_part_l, nparts,
                                                               (float)(1.0 / (3.0 * nb)), h->mlp_grad, loss_dst);
  HIP_TRY(hipGetLastError());
  return LB_OK;
}

int lb_mlp_gradient(lb_handle* h, const float* rows, const float* targets, long long m, float* grad, float* loss) {
  if (!h || !rows || !targets || !grad || !loss) return fail(LB_EINVAL, "NULL argument");
  if (m < 1 || m > LB_MLP_MAX_BATCH) return fail(LB_EINVAL, "m must lie in [1, %d]", LB_MLP_MAX_BATCH);
  if (!h->mlp_weights) return fail(LB_EINVAL, "no network parameters set");
  (void)hipSetDevice(h->device);
  HIP_TRY(hipMemsetAsync(h->mlp_bad, 0, sizeof(uint32_t), h->stream));
  int rc = mlp_fwdbwd(h, rows, targets, m, nullptr, (int)m, loss);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(grad, h->mlp_grad, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LB_OK;
}

int lb_mlp_train(lb_handle* h, const float* rows, const float* targets, long long m, const int* order, int n_steps,
                 int batch, double lr, float* loss_log) {
  if (!h || !rows || !targets || (!order && n_steps > 0)) return fail(LB_EINVAL, "NULL argument");
  if (m < 1) return fail(LB_EINVAL, "m must be >= 1");
  if (n_steps < 0) return fail(LB_EINVAL, "n_steps must be >= 0");
  if (batch < 1 || batch > LB_MLP_MAX_BATCH) return fail(LB_EINVAL, "batch must lie in [1, %d]", LB_MLP_MAX_BATCH);
  if (!(lr > 0.0) || !std::isfinite(lr)) return fail(LB_EINVAL, "lr must be positive");
  if (!h->mlp_weights) return fail(LB_EINVAL, "set initial network parameters first (lb_mlp_set_weights)");
  (void)hipSetDevice(h->device);
  HIP_TRY(hipMemsetAsync(h->mlp_bad, 0, sizeof(uint32_t), h->stream));
  HIP_TRY(hipMemsetAsync(h->mlp_m1, 0, sizeof(float) * MLP_PARAMS, h->stream));
  HIP_TRY(hipMemsetAsync(h->mlp_m2, 0, sizeof(float) * MLP_PARAMS, h->stream));
  double p1 = 1.0, p2 = 1.0;
  for (int t = 0; t < n_steps; ++t) {
    int rc = mlp_fwdbwd(h, rows, targets, m, order + (size_t)t * batch, batch,
                        loss_log ? loss_log + t : h->mlp_grad + MLP_PARAMS);
    if (rc) return rc;
    p1 *= 0.9;
    p2 *= 0.999;
    k_mlp_adam<<<(MLP_PARAMS + 255) / 256, 256, 0, h->stream>>>(h->mlp_theta, h->mlp_m1, h->mlp_m2, h->mlp_grad,
                                                                (float)lr, (float)(1.0 - p1), (float)(1.0 - p2));
    HIP_TRY(hipGetLastError());
  }
  // input ranges of the training rows
  const int nparts = (int)std::min<long long>(1024, (m + 7) / 8);
  float* part = nullptr;
  int rc = dev_alloc((void**)&part, sizeof(float) * 64 * (size_t)nparts, "range partials");
  if (rc) return rc;
  k_mlp_range_part<<<nparts, 256, 0, h->stream>>>(rows, m, part);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    k_mlp_range_final<<<1, 32, 0, h->stream>>>(part, nparts, h->mlp_lo, h->mlp_lo + 32);
    e = hipGetLastError();
  }
  float r[64];
  uint32_t bad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(r, h->mlp_lo, sizeof r, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, h->mlp_bad, sizeof bad, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(part);
  if (e != hipSuccess) return fail(LB_EHIP, "closure training: %s", hipGetErrorString(e));
  // column 30 holds |g|: its minimum is the smallest training |g|
  h->mlp_gmin = r[MLP_IN];
  for (int k = MLP_IN; k < 32; ++k) {
    r[k] = INFINITY;
    r[32 + k] = -INFINITY;
  }
  HIP_TRY(hipMemcpyAsync(h->mlp_lo, r, sizeof r, hipMemcpyHostToDevice, h->stream));
  if ((rc = mlp_pack(h))) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (bad) return fail(LB_EINVAL, "order holds row indices outside [0, %lld); those rows were skipped", m);
  return LB_OK;
}

int lb_mlp_infer(lb_handle* h, const float* rows, float* out, long long m) {
  if (!h || (m > 0 && (!rows || !out))) return fail(LB_EINVAL, "NULL argument");
  if (m < 0) return fail(LB_EINVAL, "m must be >= 0");
  if (!h->mlp_weights) return fail(LB_EINVAL, "no network parameters set");
  if (m == 0) return LB_OK;
  (void)hipSetDevice(h->device);
  const long long blocks = (m + 63) / 64;
  if (blocks > 0x7fffffffLL) return fail(LB_EINVAL, "too many rows");
  k_mlp_infer<<<(unsigned)blocks, 256, 0, h->stream>>>(h->mlp_net, rows, m, out);
  HIP_TRY(hipGetLastError());
  return LB_OK;
}

}  // extern "C"

template <class L, class R>
static int collect_t(lb_handle* h, float* rows, float* targets, long long cap, long long* m_active, long long* m_free) {
  CollectArgs a{};
  a.nx = h->p.nx; a.ny = h->p.ny; a.nz = h->p.nz;
  a.wall_x = h->p.wall[0]; a.wall_y = h->p.wall[1]; a.wall_z = h->p.wall[2];
  a.N = h->N;
  a.phi_I = h->p.phi_interface;
  a.inv_ncA = 1.0 / h->p.nc_A;
  const uint32_t nblk = (h->N + 255) / 256;
  uint32_t* counts = nullptr;
  uint64_t* offs = nullptr;
  int rc = dev_alloc((void**)&counts, sizeof(uint32_t) * 2 * nblk, "collection counts");
  if (rc) return rc;
  if ((rc = dev_alloc((void**)&offs, sizeof(uint64_t) * 2 * nblk, "collection offsets"))) {
    (void)hipFree(counts);
    return rc;
  }
  std::vector<uint32_t> c(2 * (size_t)nblk);
  std::vector<uint64_t> o(2 * (size_t)nblk);
  const R* phi = (const R*)h->phi_field();
  const R* fnc = (const R*)h->fnc;
  hipError_t e = hipSuccess;
  k_collect_count<L, R><<<nblk, 256, 0, h->stream>>>(phi, fnc, a, counts);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(c.data(), counts, sizeof(uint32_t) * c.size(), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  uint64_t na = 0, nf = 0;
  if (e == hipSuccess) {
    for (uint32_t b = 0; b < nblk; ++b) na += c[2 * b];
    uint64_t ra = 0, rf = na;
    for (uint32_t b = 0; b < nblk; ++b) {
      o[2 * b] = ra;
      o[2 * b + 1] = rf;
      ra += c[2 * b];
      rf += c[2 * b + 1];
    }
    nf = rf - na;
    e = hipMemcpyAsync(offs, o.data(), sizeof(uint64_t) * o.size(), hipMemcpyHostToDevice, h->stream);
  }
  if (e == hipSuccess && cap > 0) {
    k_collect_write<L, R><<<nblk, 256, 0, h->stream>>>(phi, fnc, a, offs, cap, rows, targets);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(counts);
  (void)hipFree(offs);
  if (e != hipSuccess) return fail(LB_EHIP, "closure row collection: %s", hipGetErrorString(e));
  *m_active = (long long)na;
  *m_free = (long long)nf;
  return LB_OK;
}

// ------------------------------------------------ allocation-free collection
// Scratch of lb_nc_collect_noalloc: per-workgroup counts (2 x uint32 per
// workgroup of 256 sites, packed two per uint64 element), their offsets
// (2 x uint64 per workgroup) and the two totals, for lattices of up to
// COLLECT_MAX_BLOCKS x 256 sites.  Each GPU holds its own copy; host code
// reaches it only through the address hipGetSymbolAddress gives on that
// device (collect_scratch_ptr).
constexpr uint32_t COLLECT_MAX_BLOCKS = 1u << 18;  // 67,108,864 sites
constexpr size_t COLLECT_SCRATCH_WORDS = (size_t)COLLECT_MAX_BLOCKS + 2 * (size_t)COLLECT_MAX_BLOCKS + 2;
static __device__ __align__(256) uint64_t scratch[COLLECT_SCRATCH_WORDS];

namespace {
constexpr int MAX_DEVICES = 64;
void* g_scratch_ptr[MAX_DEVICES] = {};
std::mutex g_scratch_mu;
}  // namespace

// the device address of this GPU's scratch array (looked up once per device,
// with that device current)
static int collect_scratch_ptr(int device, uint64_t** out) {
  if (device < 0 || device >= MAX_DEVICES) return fail(LB_EUNSUPPORTED, "device index %d beyond %d", device, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(LB_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = (uint64_t*)g_scratch_ptr[device];
  return LB_OK;
}

template <class L, class R>
static int collect_noalloc_t(lb_handle* h, float* rows, float* targets, long long cap, long long* m_active,
                             long long* m_free) {
  CollectArgs a{};
  a.nx = h->p.nx; a.ny = h->p.ny; a.nz = h->p.nz;
  a.wall_x = h->p.wall[0]; a.wall_y = h->p.wall[1]; a.wall_z = h->p.wall[2];
  a.N = h->N;
  a.phi_I = h->p.phi_interface;
  a.inv_ncA = 1.0 / h->p.nc_A;
  const uint32_t nblk = (h->N + 255) / 256;
  uint64_t* base = nullptr;
  int rc = collect_scratch_ptr(h->device, &base);
  if (rc) return rc;
  uint32_t* counts = (uint32_t*)base;                       // 2 x nblk uint32
  uint64_t* offs = base + COLLECT_MAX_BLOCKS;               // 2 x nblk uint64
  uint64_t* totals = offs + 2 * (size_t)COLLECT_MAX_BLOCKS;  // 2 uint64
  const R* phi = (const R*)h->phi_field();
  const R* fnc = (const R*)h->fnc;
  // every entry the kernels read is written first in this call: counts and
  // offsets of workgroups 0 .. nblk-1, and the totals
  k_collect_count<L, R><<<nblk, 256, 0, h->stream>>>(phi, fnc, a, counts);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    k_collect_scan<<<1, 1024, 0, h->stream>>>(counts, nblk, offs, totals);
    e = hipGetLastError();
  }
  if (e == hipSuccess && cap > 0) {
    k_collect_write<L, R><<<nblk, 256, 0, h->stream>>>(phi, fnc, a, offs, cap, rows, targets);
    e = hipGetLastError();
  }
  uint64_t tot[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(tot, totals, sizeof tot, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(LB_EHIP, "closure row collection: %s", hipGetErrorString(e));
  *m_active = (long long)tot[0];
  *m_free = (long long)tot[1];
  return LB_OK;
}

extern "C" {

int lb_nc_collect_noalloc(lb_handle* h, int channel, float* rows, float* targets, long long cap,
                          long long* m_active, long long* m_free) {
  if (!h || !m_active || !m_free) return fail(LB_EINVAL, "NULL argument");
  if (h->ensemble()) {
    if (channel < 0 || channel >= (int)h->chans.size()) return fail(LB_EINVAL, "channel %d out of range", channel);
    return lb_nc_collect_noalloc(h->chans[channel], 0, rows, targets, cap, m_active, m_free);
  }
  if (channel != 0) return fail(LB_EINVAL, "channel %d out of range", channel);
  if (cap < 0 || (cap > 0 && (!rows || !targets))) return fail(LB_EINVAL, "bad output buffers");
  if (h->d != 3) return fail(LB_EINVAL, "the learned closure is 3D only");
  if (h->p.nc_mode != LB_NC_EXPLICIT) return fail(LB_EINVAL, "collection needs a step with LB_NC_EXPLICIT");
  if (!h->fields_valid || h->t == 0) return fail(LB_EINVAL, "take a step first: rows come from the last step");
  if ((h->N + 255) / 256 > COLLECT_MAX_BLOCKS)
    return fail(LB_EINVAL, "%u sites: the allocation-free collection takes at most %u sites (its static scratch)",
                h->N, COLLECT_MAX_BLOCKS * 256u);
  (void)hipSetDevice(h->device);
  const bool f64 = h->p.storage == LB_F64;
  if (h->p.lattice == LB_D3Q19)
    return f64 ? collect_noalloc_t<D3Q19, double>(h, rows, targets, cap, m_active, m_free)
               : collect_noalloc_t<D3Q19, float>(h, rows, targets, cap, m_active, m_free);
  return f64 ? collect_noalloc_t<D3Q27, double>(h, rows, targets, cap, m_active, m_free)
             : collect_noalloc_t<D3Q27, float>(h, rows, targets, cap, m_active, m_free);
}

int lb_nc_collect(lb_handle* h, int channel, float* rows, float* targets, long long cap, long long* m_active,
                  long long* m_free) {
  if (!h || !m_active || !m_free) return fail(LB_EINVAL, "NULL argument");
  if (h->ensemble()) {
    if (channel < 0 || channel >= (int)h->chans.size()) return fail(LB_EINVAL, "channel %d out of range", channel);
    return lb_nc_collect(h->chans[channel], 0, rows, targets, cap, m_active, m_free);
  }
  if (channel != 0) return fail(LB_EINVAL, "channel %d out of range", channel);
  if (cap < 0 || (cap > 0 && (!rows || !targets))) return fail(LB_EINVAL, "bad output buffers");
  if (h->d != 3) return fail(LB_EINVAL, "the learned closure is 3D only");
  if (h->p.nc_mode != LB_NC_EXPLICIT) return fail(LB_EINVAL, "collection needs a step with LB_NC_EXPLICIT");
  if (!h->fields_valid || h->t == 0) return fail(LB_EINVAL, "take a step first: rows come from the last step");
  (void)hipSetDevice(h->device);
  const bool f64 = h->p.storage == LB_F64;
  if (h->p.lattice == LB_D3Q19)
    return f64 ? collect_t<D3Q19, double>(h, rows, targets, cap, m_active, m_free)
               : collect_t<D3Q19, float>(h, rows, targets, cap, m_active, m_free);
  return f64 ? collect_t<D3Q27, double>(h, rows, targets, cap, m_active, m_free)
             : collect_t<D3Q27, float>(h, rows, targets, cap, m_active, m_free);
}

}  // extern "C"
