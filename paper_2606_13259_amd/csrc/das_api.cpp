// C-ABI layer of the delay-and-sum library: plan lifetime, host-side
// validation, algorithm choice, workspace sizing and kernel dispatch.
// Every entry point returns das_status; failures leave a thread-local message
// for das_last_error().  Arguments are validated before any HIP call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "das.h"
#include "das_internal.h"

using namespace dasmi;

namespace {

thread_local std::string g_last_error;

das_status fail(das_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

das_status hip_fail(hipError_t e, const char* what) {
  return fail(DAS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Candidate 256-voxel tiles of the windowed kernel (the autotuner's space).
const int kTiles[][3] = {{8, 8, 4}, {16, 4, 4}, {4, 8, 8}, {16, 8, 2},
                         {8, 4, 8}, {16, 16, 1}, {32, 8, 1}, {4, 4, 16}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
// Counter sets per plan for persistent MFMA launches (launches of one plan
// that overlap on different streams: at most this many).
constexpr unsigned kCounterSets = 64;

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

TileShape tile_shape(int idx) {
  TileShape t;
  t.tx = kTiles[idx][0];
  t.ty = kTiles[idx][1];
  t.tz = kTiles[idx][2];
  t.lx = ilog2(t.tx);
  t.lxy = ilog2(t.tx * t.ty);
  // wavefront box: halve the longest side (z, then x, then y on ties) until
  // 64 voxels remain
  int w[3] = {t.tx, t.ty, t.tz};
  while (w[0] * w[1] * w[2] > 64) {
    int d = 2;
    if (w[0] > w[d]) d = 0;
    if (w[1] > w[d]) d = 1;
    w[d] /= 2;
  }
  t.wx = w[0];
  t.wy = w[1];
  t.wz = w[2];
  t.wlx = ilog2(t.wx);
  t.wlxy = ilog2(t.wx * t.wy);
  t.bx = t.tx / t.wx;
  t.by = t.ty / t.wy;
  t.blx = ilog2(t.bx);
  t.blxy = ilog2(t.bx * t.by);
  return t;
}

constexpr size_t kMaxLds = 160 * 1024;

// RAII: make the plan's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

bool finite3(const double* v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

}  // namespace

namespace dasmi {

int tiled_batch_per_thread(int storage, int B) {
  (void)storage;
  if (B >= 4) return 4;
  if (B >= 2) return 2;
  return 1;
}

size_t tiled_lds_bytes(const Geom& g, int storage, int bt, const Window& w) {
  if (storage == DAS_STORE_F32) return tiled_lds_f32(g, bt, w);
  if (storage == DAS_STORE_F16) return tiled_lds_f16(g, bt, w);
  if (storage == DAS_STORE_FP8_E4M3) return tiled_lds_fp8(g, bt, w);
  return tiled_lds_bf16(g, bt, w);
}

hipError_t launch_tiled_forward(const Geom& g, int storage, const TileShape& ts, const Window& w,
                                const void* ws, int B, float* x, hipStream_t st) {
  if (storage == DAS_STORE_F32) return tiled_forward_f32(g, ts, w, ws, B, x, st);
  if (storage == DAS_STORE_F16) return tiled_forward_f16(g, ts, w, ws, B, x, st);
  if (storage == DAS_STORE_FP8_E4M3) return tiled_forward_fp8(g, ts, w, ws, B, x, st);
  return tiled_forward_bf16(g, ts, w, ws, B, x, st);
}

}  // namespace dasmi

struct das_plan_s {
  int device = 0;
  das_config cfg{};
  int M = 0, Q = 0, K = 0, N = 0;
  double c = 0.0;
  double* d_elem = nullptr;
  float* d_norm = nullptr;
  double* d_txvec = nullptr;
  double* d_txoff = nullptr;
  int* d_txkind = nullptr;
  // Work counters of persistent MFMA launches led by this plan: kCounterSets
  // sets used in turn, so that launches that overlap on different streams use
  // different sets.
  unsigned* d_ctr = nullptr;
  std::atomic<unsigned> ctr_next{0};
  const float* w_tx = nullptr;
  int algo = DAS_ALGO_AUTO;  // forced algorithm (AUTO = choose)
  int tile = 0;              // index into kTiles
  bool has_diverging = false;
  // Whether AUTO uses the windowed (batch-inner) workspace layout; fixed at
  // plan creation so that the layout written by das_prepare and read by
  // das_forward never depends on later tile or sound-speed changes.
  bool auto_tiled = false;
  // Complex baseband mode (das_plan_set_iq): carrier frequency (Hz).
  bool iq = false;
  double fc = 0.0;
  int interp = DAS_INTERP_LINEAR;  // das_plan_set_interp
  int mfma_form = DAS_MFMA_AUTO;  // das_plan_set_mfma_form
};

namespace {

Geom make_geom(const das_plan_s* p) {
  Geom g{};
  g.elem = p->d_elem;
  g.enorm = p->d_norm;
  g.txvec = p->d_txvec;
  g.txoff = p->d_txoff;
  g.txkind = p->d_txkind;
  g.w_tx = p->w_tx;
  for (int i = 0; i < 3; ++i) {
    g.o[i] = p->cfg.grid.origin[i];
    g.s[i] = p->cfg.grid.spacing[i];
    g.n[i] = p->cfg.grid.dims[i];
  }
  g.M = p->M;
  g.Q = p->Q;
  g.K = p->K;
  g.c = p->c;
  g.fs = p->cfg.fs;
  g.fsc = p->cfg.fs / p->c;
  g.t0fs = p->cfg.t0 * p->cfg.fs;
  g.apod = p->cfg.apod;
  g.fourF2 = (float)(4.0 * p->cfg.f_number * p->cfg.f_number);
  g.iq = p->iq ? 1 : 0;
  g.fcfs = p->iq ? p->fc / p->cfg.fs : 0.0;
  const double ft = p->iq ? p->fc * p->cfg.t0 : 0.0;
  g.fct0 = ft - std::floor(ft);
  return g;
}

// Window of a tile shape at the plan's current sound speed: every voxel of the
// tile has |f - (ktx + krx)| < 2 D + 1 where D = |half diagonal| * fs / c
// (both path differences are bounded by |dp| by the triangle inequality).
Window make_window(const das_plan_s* p, const TileShape& ts) {
  const double hx = 0.5 * (ts.tx - 1) * p->cfg.grid.spacing[0];
  const double hy = 0.5 * (ts.ty - 1) * p->cfg.grid.spacing[1];
  const double hz = 0.5 * (ts.tz - 1) * p->cfg.grid.spacing[2];
  const double D = std::sqrt(hx * hx + hy * hy + hz * hz) * (p->cfg.fs / p->c);
  Window w;
  w.dint = (int)std::ceil(2.0 * D * (1.0 + 1e-6)) + 1;
  w.pairs = 2 * w.dint + 3;
  return w;
}

bool tiled_fits(const das_plan_s* p, int tile, int B) {
  const Geom g = make_geom(p);
  const Window w = make_window(p, tile_shape(tile));
  const int st = p->cfg.storage;
  const int bt = tiled_batch_per_thread(st, B);
  const size_t lds = tiled_lds_bytes(g, st, bt, w);
  // one lane per window sample
  return lds > 0 && lds <= kMaxLds && w.pairs + 1 <= 64;
}

hipError_t launch_windowed(const das_plan_s* p, const Geom& g, int tile, const void* ws, int B,
                           float* x, hipStream_t st) {
  const TileShape ts = tile_shape(tile);
  const Window w = make_window(p, ts);
  if (p->iq) return tiled_forward_f32_iq(g, ts, w, ws, B, x, st);
  if (p->interp == DAS_INTERP_CUBIC) return tiled_forward_f32_cubic(g, ts, w, ws, B, x, st);
  return launch_tiled_forward(g, p->cfg.storage, ts, w, ws, B, x, st);
}

// The algorithm, and with it the workspace layout, depends only on the forced
// algorithm and on what was decided at plan creation -- never on the current
// tile or sound speed -- so das_prepare and das_forward always agree.
// Batch size from which AUTO contracts on the matrix cores (16- or 8-bit storage).
constexpr int kMfmaMinBatch = 16;

int choose_algo(const das_plan_s* p, int B) {
  if (p->algo != DAS_ALGO_AUTO) return p->algo;
  if (p->cfg.storage != DAS_STORE_F32 && B >= kMfmaMinBatch) return DAS_ALGO_MFMA;
  return p->auto_tiled ? DAS_ALGO_TILED : DAS_ALGO_PLAIN;
}

size_t storage_bytes(int storage) {
  return storage == DAS_STORE_F32 ? 4 : storage == DAS_STORE_FP8_E4M3 ? 1 : 2;
}

// Bytes of the samples of a workspace for B items.
size_t ws_data_bytes(const das_plan_s* p, int B) {
  const int algo = choose_algo(p, B);
  const size_t elems = (size_t)B * p->Q * p->M * p->K;
  if (algo == DAS_ALGO_PLAIN) return elems * 4;
  if (algo == DAS_ALGO_MFMA) return mfma_workspace_elems(make_geom(p), B) * storage_bytes(p->cfg.storage);
  return elems * storage_bytes(p->cfg.storage);
}

// FP8 workspaces (windowed or MFMA layout) end with the per-item scale table:
// B f32 values at the first 256-byte boundary after the samples.
bool has_fp8_table(const das_plan_s* p, int B) {
  return p->cfg.storage == DAS_STORE_FP8_E4M3 && choose_algo(p, B) != DAS_ALGO_PLAIN;
}
size_t fp8_table_offset(const das_plan_s* p, int B) { return (ws_data_bytes(p, B) + 255) & ~(size_t)255; }

size_t ws_bytes(const das_plan_s* p, int B) {
  if (has_fp8_table(p, B)) return fp8_table_offset(p, B) + sizeof(float) * (size_t)B;
  return ws_data_bytes(p, B);
}

// The geometry of a call on workspace ws of B items (with the FP8 scale table).
Geom call_geom(const das_plan_s* p, const void* ws, int B) {
  Geom g = make_geom(p);
  if (has_fp8_table(p, B))
    g.amax = reinterpret_cast<const float*>(static_cast<const char*>(ws) + fp8_table_offset(p, B));
  return g;
}

das_status check_plan(das_plan p) {
  if (!p) return fail(DAS_ERR_INVALID_ARG, "plan is NULL");
  return DAS_OK;
}

das_status check_batch(das_plan p, int32_t batch) {
  if (batch < 1 || batch > p->cfg.max_batch)
    return fail(DAS_ERR_INVALID_ARG, "batch " + std::to_string(batch) + " outside [1, max_batch=" +
                                         std::to_string(p->cfg.max_batch) + "]");
  return DAS_OK;
}

}  // namespace

extern "C" {

const char* das_version(void) { return "das-mi355x 0.1 (gfx950)"; }

const char* das_status_string(das_status st) {
  switch (st) {
    case DAS_OK: return "DAS_OK";
    case DAS_ERR_INVALID_ARG: return "DAS_ERR_INVALID_ARG";
    case DAS_ERR_UNSUPPORTED: return "DAS_ERR_UNSUPPORTED";
    case DAS_ERR_HIP: return "DAS_ERR_HIP";
    case DAS_ERR_OOM: return "DAS_ERR_OOM";
  }
  return "DAS_ERR_UNKNOWN";
}

const char* das_last_error(void) { return g_last_error.c_str(); }

int32_t das_num_tile_shapes(void) { return kNumTiles; }

das_status das_tile_shape(int32_t idx, int32_t dims[3]) {
  if (idx < 0 || idx >= kNumTiles || !dims) return fail(DAS_ERR_INVALID_ARG, "bad tile index");
  for (int i = 0; i < 3; ++i) dims[i] = kTiles[idx][i];
  return DAS_OK;
}

das_status das_plan_create(das_plan* out, const das_config* cfg, int hip_device) {
  if (!out) return fail(DAS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(DAS_ERR_INVALID_ARG, "cfg is NULL");
  const int M = cfg->num_elements, Q = cfg->num_tx, K = cfg->num_samples;
  if (M < 1 || M > 65535) return fail(DAS_ERR_INVALID_ARG, "num_elements must be in [1, 65535]");
  if (Q < 1 || Q > 4096) return fail(DAS_ERR_INVALID_ARG, "num_tx must be in [1, 4096]");
  if (K < 2) return fail(DAS_ERR_INVALID_ARG, "num_samples must be >= 2");
  if (!cfg->element_pos) return fail(DAS_ERR_INVALID_ARG, "element_pos is NULL");
  if (!cfg->tx) return fail(DAS_ERR_INVALID_ARG, "tx is NULL");
  long long N = 1;
  for (int i = 0; i < 3; ++i) {
    if (cfg->grid.dims[i] < 1) return fail(DAS_ERR_INVALID_ARG, "grid dims must be >= 1");
    if (!(cfg->grid.spacing[i] > 0.0) || !std::isfinite(cfg->grid.spacing[i]))
      return fail(DAS_ERR_INVALID_ARG, "grid spacing must be finite and > 0");
    if (!std::isfinite(cfg->grid.origin[i])) return fail(DAS_ERR_INVALID_ARG, "grid origin not finite");
    N *= cfg->grid.dims[i];
  }
  if (N > (1ll << 31) - 1) return fail(DAS_ERR_INVALID_ARG, "more than 2^31-1 voxels");
  if (!(cfg->sound_speed > 0.0) || !std::isfinite(cfg->sound_speed))
    return fail(DAS_ERR_INVALID_ARG, "sound_speed must be finite and > 0");
  if (!(cfg->fs > 0.0) || !std::isfinite(cfg->fs)) return fail(DAS_ERR_INVALID_ARG, "fs must be finite and > 0");
  if (!std::isfinite(cfg->t0)) return fail(DAS_ERR_INVALID_ARG, "t0 not finite");
  if (cfg->max_batch < 1) return fail(DAS_ERR_INVALID_ARG, "max_batch must be >= 1");
  if (cfg->apod != DAS_APOD_UNIFORM && cfg->apod != DAS_APOD_HANN_FNUM)
    return fail(DAS_ERR_INVALID_ARG, "unknown apod");
  if (cfg->apod == DAS_APOD_HANN_FNUM && !(cfg->f_number > 0.0 && std::isfinite(cfg->f_number)))
    return fail(DAS_ERR_INVALID_ARG, "f_number must be finite and > 0");
  if (cfg->storage < DAS_STORE_F32 || cfg->storage > DAS_STORE_FP8_E4M3)
    return fail(DAS_ERR_INVALID_ARG, "unknown storage");
  if (cfg->algo < DAS_ALGO_AUTO || cfg->algo > DAS_ALGO_MFMA)
    return fail(DAS_ERR_INVALID_ARG, "unknown algo");
  if (cfg->algo == DAS_ALGO_MFMA && cfg->storage == DAS_STORE_F32)
    return fail(DAS_ERR_UNSUPPORTED, "the MFMA form needs f16, bf16 or fp8 storage");
  for (int m = 0; m < M; ++m)
    if (!finite3(cfg->element_pos + 3 * m)) return fail(DAS_ERR_INVALID_ARG, "element_pos not finite");
  std::vector<float> norm;
  if (cfg->element_normal) {
    norm.resize(3 * (size_t)M);
    for (int m = 0; m < M; ++m) {
      const double* v = cfg->element_normal + 3 * m;
      const double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      if (!finite3(v) || !(l > 0.0)) return fail(DAS_ERR_INVALID_ARG, "element_normal must be nonzero and finite");
      for (int i = 0; i < 3; ++i) norm[3 * m + i] = (float)(v[i] / l);
    }
  }
  std::vector<double> txvec(3 * (size_t)Q), txoff(Q);
  std::vector<int> txkind(Q);
  bool diverging = false;
  for (int q = 0; q < Q; ++q) {
    const das_tx& t = cfg->tx[q];
    if (t.kind != DAS_TX_NONE && t.kind != DAS_TX_PLANE && t.kind != DAS_TX_DIVERGING)
      return fail(DAS_ERR_INVALID_ARG, "unknown transmit kind");
    if (!finite3(t.vec) || !std::isfinite(t.path_offset))
      return fail(DAS_ERR_INVALID_ARG, "transmit descriptor not finite");
    if (t.kind == DAS_TX_PLANE) {
      const double l = std::sqrt(t.vec[0] * t.vec[0] + t.vec[1] * t.vec[1] + t.vec[2] * t.vec[2]);
      if (std::fabs(l - 1.0) > 1e-6) return fail(DAS_ERR_INVALID_ARG, "plane-wave direction must be a unit vector");
    }
    diverging |= t.kind == DAS_TX_DIVERGING;
    for (int i = 0; i < 3; ++i) txvec[3 * q + i] = t.vec[i];
    txoff[q] = t.path_offset;
    txkind[q] = t.kind;
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= ndev) return fail(DAS_ERR_INVALID_ARG, "bad hip_device");

  das_plan_s* p = new das_plan_s();
  p->device = hip_device;
  p->cfg = *cfg;
  p->cfg.element_pos = nullptr;
  p->cfg.element_normal = nullptr;
  p->cfg.tx = nullptr;
  p->M = M;
  p->Q = Q;
  p->K = K;
  p->N = (int)N;
  p->c = cfg->sound_speed;
  p->algo = cfg->algo;
  p->has_diverging = diverging;
  DeviceGuard dg(hip_device);
  if (!dg.ok) {
    delete p;
    return fail(DAS_ERR_HIP, "hipSetDevice failed");
  }
  auto alloc_copy = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t r = hipMalloc(dst, bytes);
    if (r != hipSuccess) return r;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  e = alloc_copy((void**)&p->d_elem, cfg->element_pos, sizeof(double) * 3 * M);
  if (e == hipSuccess && !norm.empty()) e = alloc_copy((void**)&p->d_norm, norm.data(), sizeof(float) * 3 * M);
  if (e == hipSuccess) e = alloc_copy((void**)&p->d_txvec, txvec.data(), sizeof(double) * 3 * Q);
  if (e == hipSuccess) e = alloc_copy((void**)&p->d_txoff, txoff.data(), sizeof(double) * Q);
  if (e == hipSuccess) e = alloc_copy((void**)&p->d_txkind, txkind.data(), sizeof(int) * Q);
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_ctr, kCounterSets * mfma_batched_counter_bytes());
  if (e != hipSuccess) {
    das_plan_destroy(p);
    return e == hipErrorOutOfMemory ? fail(DAS_ERR_OOM, "hipMalloc failed") : hip_fail(e, "plan upload");
  }
  for (int ti = 0; ti < kNumTiles; ++ti) {
    if (tiled_fits(p, ti, 1)) {
      p->auto_tiled = true;
      p->tile = ti;
      break;
    }
  }
  *out = p;
  return DAS_OK;
}

das_status das_plan_destroy(das_plan p) {
  if (!p) return DAS_OK;
  DeviceGuard dg(p->device);
  (void)hipDeviceSynchronize();
  if (p->d_elem) (void)hipFree(p->d_elem);
  if (p->d_norm) (void)hipFree(p->d_norm);
  if (p->d_txvec) (void)hipFree(p->d_txvec);
  if (p->d_txoff) (void)hipFree(p->d_txoff);
  if (p->d_txkind) (void)hipFree(p->d_txkind);
  if (p->d_ctr) (void)hipFree(p->d_ctr);
  delete p;
  return DAS_OK;
}

das_status das_plan_set_sound_speed(das_plan p, double c) {
  if (das_status s = check_plan(p)) return s;
  if (!(c > 0.0) || !std::isfinite(c)) return fail(DAS_ERR_INVALID_ARG, "sound speed must be finite and > 0");
  p->c = c;
  return DAS_OK;
}

das_status das_plan_set_tx_weights(das_plan p, const float* w_tx) {
  if (das_status s = check_plan(p)) return s;
  p->w_tx = w_tx;
  return DAS_OK;
}

das_status das_plan_set_algo(das_plan p, int32_t algo) {
  if (das_status s = check_plan(p)) return s;
  if (algo < DAS_ALGO_AUTO || algo > DAS_ALGO_MFMA) return fail(DAS_ERR_INVALID_ARG, "unknown algo");
  if (algo == DAS_ALGO_MFMA && p->cfg.storage == DAS_STORE_F32)
    return fail(DAS_ERR_UNSUPPORTED, "the MFMA form needs f16, bf16 or fp8 storage");
  if (p->interp == DAS_INTERP_CUBIC && (algo == DAS_ALGO_PLAIN || algo == DAS_ALGO_MFMA ||
                                        (algo == DAS_ALGO_AUTO && !p->auto_tiled)))
    return fail(DAS_ERR_UNSUPPORTED, "cubic interpolation runs in the windowed algorithm only");
  p->algo = algo;
  return DAS_OK;
}

das_status das_plan_set_mfma_form(das_plan p, int32_t form) {
  if (das_status s = check_plan(p)) return s;
  if (form < DAS_MFMA_AUTO || form > DAS_MFMA_SLAB_FP8)
    return fail(DAS_ERR_INVALID_ARG, "unknown MFMA form");
  if ((form == DAS_MFMA_COLUMN_FP8 || form == DAS_MFMA_SLAB_FP8) &&
      p->cfg.storage != DAS_STORE_FP8_E4M3)
    return fail(DAS_ERR_UNSUPPORTED, "FP8 matrix operands need FP8 storage");
  p->mfma_form = form;
  return DAS_OK;
}

das_status das_plan_get_mfma_form(das_plan p, int32_t* form) {
  if (das_status s = check_plan(p)) return s;
  if (!form) return fail(DAS_ERR_INVALID_ARG, "form is NULL");
  *form = p->mfma_form;
  return DAS_OK;
}

das_status das_plan_set_interp(das_plan p, int32_t interp) {
  if (das_status s = check_plan(p)) return s;
  if (interp != DAS_INTERP_LINEAR && interp != DAS_INTERP_CUBIC)
    return fail(DAS_ERR_INVALID_ARG, "unknown interpolation");
  if (interp == DAS_INTERP_CUBIC) {
    if (p->cfg.storage != DAS_STORE_F32)
      return fail(DAS_ERR_UNSUPPORTED, "cubic interpolation runs with f32 storage only");
    const bool tiled = p->algo == DAS_ALGO_TILED || (p->algo == DAS_ALGO_AUTO && p->auto_tiled);
    if (!tiled)
      return fail(DAS_ERR_UNSUPPORTED, "cubic interpolation runs in the windowed algorithm only");
  }
  p->interp = interp;
  return DAS_OK;
}

das_status das_plan_get_algo(das_plan p, int32_t batch, int32_t* algo) {
  if (das_status s = check_plan(p)) return s;
  if (!algo) return fail(DAS_ERR_INVALID_ARG, "algo is NULL");
  if (das_status s = check_batch(p, batch)) return s;
  *algo = choose_algo(p, batch);
  return DAS_OK;
}

das_status das_plan_get_tile(das_plan p, int32_t* tile_index) {
  if (das_status s = check_plan(p)) return s;
  if (!tile_index) return fail(DAS_ERR_INVALID_ARG, "tile_index is NULL");
  *tile_index = p->tile;
  return DAS_OK;
}

das_status das_plan_set_iq(das_plan p, int32_t enable, double fc) {
  if (das_status s = check_plan(p)) return s;
  if (!std::isfinite(fc) || fc < 0.0) return fail(DAS_ERR_INVALID_ARG, "fc must be finite and >= 0");
  p->iq = enable != 0;
  p->fc = p->iq ? fc : 0.0;
  return DAS_OK;
}

das_status das_plan_set_tile(das_plan p, int32_t tile_index) {
  if (das_status s = check_plan(p)) return s;
  if (tile_index < 0 || tile_index >= kNumTiles) return fail(DAS_ERR_INVALID_ARG, "bad tile index");
  if (!tiled_fits(p, tile_index, 1))
    return fail(DAS_ERR_UNSUPPORTED, "the sample windows of this tile shape do not fit (one lane per sample)");
  p->tile = tile_index;
  return DAS_OK;
}

das_status das_workspace_bytes(das_plan p, int32_t batch, size_t* bytes) {
  if (das_status s = check_plan(p)) return s;
  if (!bytes) return fail(DAS_ERR_INVALID_ARG, "bytes is NULL");
  if (das_status s = check_batch(p, batch)) return s;
  *bytes = ws_bytes(p, batch);
  return DAS_OK;
}

das_status das_prepare(das_plan p, const float* y, int32_t b0, int32_t nb, int32_t batch_total,
                       void* ws, void* stream) {
  if (das_status s = check_plan(p)) return s;
  if (!y || !ws) return fail(DAS_ERR_INVALID_ARG, "y or ws is NULL");
  if (das_status s = check_batch(p, batch_total)) return s;
  if (b0 < 0 || nb < 1 || b0 + nb > batch_total)
    return fail(DAS_ERR_INVALID_ARG, "need 0 <= b0, 1 <= nb, b0 + nb <= batch_total");
  DeviceGuard dg(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Geom g = call_geom(p, ws, batch_total);
  hipError_t e;
  const int algo = choose_algo(p, batch_total);
  if (algo == DAS_ALGO_PLAIN) {
    const size_t n = (size_t)nb * p->Q * p->M * p->K;
    float* dst = static_cast<float*>(ws) + (size_t)b0 * p->Q * p->M * p->K;
    e = hipMemcpyAsync(dst, y, n * sizeof(float), hipMemcpyDeviceToDevice, st);
  } else if (algo == DAS_ALGO_MFMA) {
    e = launch_mfma_reorder(g, p->cfg.storage, y, b0, nb, batch_total, ws, st);
  } else {
    e = launch_reorder(g, p->cfg.storage, y, b0, nb, batch_total, ws, st);
  }
  if (e != hipSuccess) return hip_fail(e, "das_prepare launch");
  return DAS_OK;
}

static das_status forward_batched_mfma(int32_t count, const das_plan* plans, const void* const* ws,
                                       const int32_t* batch, float* const* x, void* stream);

das_status das_forward(das_plan p, const void* ws, int32_t batch, float* x, void* stream) {
  if (das_status s = check_plan(p)) return s;
  if (!ws || !x) return fail(DAS_ERR_INVALID_ARG, "ws or x is NULL");
  if (das_status s = check_batch(p, batch)) return s;
  DeviceGuard dg(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Geom g = call_geom(p, ws, batch);
  const int algo = choose_algo(p, batch);
  hipError_t e = hipSuccess;
  if (p->interp == DAS_INTERP_CUBIC && (p->iq || algo != DAS_ALGO_TILED))
    return fail(DAS_ERR_UNSUPPORTED, "cubic interpolation runs in the windowed algorithm on real data");
  if (p->iq) {
    if (batch % 2) return fail(DAS_ERR_INVALID_ARG, "complex baseband needs (I, Q) pairs: an even batch");
    const bool tiled_ok = algo == DAS_ALGO_TILED && p->cfg.storage == DAS_STORE_F32;
    const bool mfma_ok = algo == DAS_ALGO_MFMA && (p->cfg.storage == DAS_STORE_F16 ||
                                                   p->cfg.storage == DAS_STORE_FP8_E4M3);
    if (!tiled_ok && !mfma_ok)
      return fail(DAS_ERR_UNSUPPORTED,
                  "complex baseband runs in the windowed algorithm with f32 storage or the MFMA "
                  "algorithm with f16 or fp8 storage");
    if (mfma_ok) {
      // persistent, column or slab launch (the FP8-operand forms are not built
      // for IQ: they fall back to the f16-operand column or slab launch)
      const int f = p->mfma_form;
      if (f == DAS_MFMA_PERSISTENT) return forward_batched_mfma(1, &p, &ws, &batch, &x, stream);
      e = launch_mfma_forward_iq(g, p->cfg.storage, ws, batch, x, f == DAS_MFMA_SLAB || f == DAS_MFMA_SLAB_FP8,
                                 st);
      if (e != hipSuccess) return hip_fail(e, "das_forward launch");
      return DAS_OK;
    }
  }
  if (algo == DAS_ALGO_PLAIN) {
    e = launch_plain_forward(g, static_cast<const float*>(ws), batch, x, st);
  } else if (algo == DAS_ALGO_TILED) {
    if (!tiled_fits(p, p->tile, batch))
      return fail(DAS_ERR_UNSUPPORTED, "tile windows do not fit in LDS for this geometry");
    e = launch_windowed(p, g, p->tile, ws, batch, x, st);
  } else if (p->mfma_form == DAS_MFMA_PERSISTENT ||
             (p->mfma_form == DAS_MFMA_AUTO && mfma_prefers_persistent(p->cfg.storage, batch))) {
    // the persistent kernel with one plan: same results, dynamic balance
    return forward_batched_mfma(1, &p, &ws, &batch, &x, stream);
  } else {
    const int f = p->mfma_form;
    e = launch_mfma_forward(g, p->cfg.storage, ws, batch, x, f == DAS_MFMA_SLAB || f == DAS_MFMA_SLAB_FP8,
                            f == DAS_MFMA_COLUMN_FP8 || f == DAS_MFMA_SLAB_FP8, st);
  }
  if (e != hipSuccess) return hip_fail(e, "das_forward launch");
  return DAS_OK;
}

das_status das_adjoint(das_plan p, const float* gx, int32_t batch, float* gy, void* stream) {
  if (das_status s = check_plan(p)) return s;
  if (p->interp != DAS_INTERP_LINEAR)
    return fail(DAS_ERR_UNSUPPORTED, "the adjoint is built for linear interpolation only");
  if (!gx || !gy) return fail(DAS_ERR_INVALID_ARG, "gx or gy is NULL");
  if (das_status s = check_batch(p, batch)) return s;
  if (p->iq && batch % 2) return fail(DAS_ERR_INVALID_ARG, "complex baseband needs an even batch");
  DeviceGuard dg(p->device);
  const Geom g = make_geom(p);
  const TileShape ts = tile_shape(p->tile);
  const Window w = make_window(p, ts);
  if (adjoint_lds_bytes(g, w) > kMaxLds)
    return fail(DAS_ERR_UNSUPPORTED, "adjoint windows do not fit in LDS");
  hipError_t e = launch_adjoint(g, ts, w, gx, batch, gy, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "das_adjoint launch");
  return DAS_OK;
}

das_status das_grad_sound_speed(das_plan p, const float* y, const float* gx, int32_t batch,
                                float* dLdc, void* stream) {
  if (das_status s = check_plan(p)) return s;
  if (p->interp != DAS_INTERP_LINEAR)
    return fail(DAS_ERR_UNSUPPORTED, "the sound-speed gradient is built for linear interpolation only");
  if (!y || !gx || !dLdc) return fail(DAS_ERR_INVALID_ARG, "y, gx or dLdc is NULL");
  if (das_status s = check_batch(p, batch)) return s;
  if (p->iq && batch % 2) return fail(DAS_ERR_INVALID_ARG, "complex baseband needs an even batch");
  DeviceGuard dg(p->device);
  hipError_t e = launch_grad_c(make_geom(p), y, gx, batch, dLdc, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "das_grad_sound_speed launch");
  return DAS_OK;
}

// Persistent MFMA launch over several plans (all validated by the caller).
static das_status forward_batched_mfma(int32_t count, const das_plan* plans, const void* const* ws,
                                       const int32_t* batch, float* const* x, void* stream) {
  MfmaBatchedArgs a{};
  a.count = count;
  for (int i = 0; i < count; ++i) {
    MfmaWork& w = a.p[i];
    w.g = call_geom(plans[i], ws[i], batch[i]);
    w.ws = ws[i];
    w.x = x[i];
    w.B = batch[i];
    w.TW = mfma_tile_width(batch[i]);
    w.Kc = mfma_chunks(w.g.K);
  }
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, plans[0]->device);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  das_plan_s* lead = plans[0];
  unsigned* ctr = lead->d_ctr + (size_t)(lead->ctr_next.fetch_add(1u) % kCounterSets) *
                                    (mfma_batched_counter_bytes() / sizeof(unsigned));
  e = launch_mfma_batched(a, ctr, lead->cfg.storage, lead->iq, cus,
                          static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "das_forward_batched launch");
  return DAS_OK;
}

das_status das_forward_batched(int32_t count, const das_plan* plans, const void* const* ws,
                               const int32_t* batch, float* const* x, void* stream) {
  if (count < 1 || !plans || !ws || !batch || !x)
    return fail(DAS_ERR_INVALID_ARG, "bad batched arguments");
  if (count > MAX_BATCHED)
    return fail(DAS_ERR_INVALID_ARG, "at most " + std::to_string(MAX_BATCHED) + " plans per launch");
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || !ws[i] || !x[i]) return fail(DAS_ERR_INVALID_ARG, "NULL entry in batched arguments");
    if (das_status s = check_batch(plans[i], batch[i])) return s;
    if (plans[i]->device != plans[0]->device)
      return fail(DAS_ERR_INVALID_ARG, "all plans of a batched launch must be on one device");
    if (plans[i]->cfg.storage != plans[0]->cfg.storage)
      return fail(DAS_ERR_UNSUPPORTED, "all plans of a batched launch must share the storage type");
    if (plans[i]->iq != plans[0]->iq)
      return fail(DAS_ERR_UNSUPPORTED, "a batched launch takes complex baseband plans only or none");
    if (plans[i]->iq && batch[i] % 2)
      return fail(DAS_ERR_INVALID_ARG, "complex baseband needs (I, Q) pairs: an even batch");
    if (plans[i]->interp != DAS_INTERP_LINEAR)
      return fail(DAS_ERR_UNSUPPORTED, "cubic-interpolation plans run through das_forward only");
  }
  const int algo0 = choose_algo(plans[0], batch[0]);
  for (int i = 0; i < count; ++i) {
    const int algo = choose_algo(plans[i], batch[i]);
    if (algo != algo0)
      return fail(DAS_ERR_UNSUPPORTED, "all plans of a batched launch must use the same algorithm");
    if (algo == DAS_ALGO_PLAIN)
      return fail(DAS_ERR_UNSUPPORTED, "batched launches need the windowed or MFMA algorithm");
    if (algo == DAS_ALGO_TILED && !tiled_fits(plans[i], plans[i]->tile, batch[i]))
      return fail(DAS_ERR_UNSUPPORTED, "tile windows do not fit for a plan of the batched launch");
  }
  DeviceGuard dg(plans[0]->device);
  const int storage = plans[0]->cfg.storage;
  if (plans[0]->iq && (algo0 != DAS_ALGO_MFMA || storage == DAS_STORE_BF16))
    return fail(DAS_ERR_UNSUPPORTED,
                "batched complex baseband launches run in the MFMA algorithm with f16 or fp8 storage");
  if (algo0 == DAS_ALGO_MFMA) return forward_batched_mfma(count, plans, ws, batch, x, stream);
  int bt = 4, qn = 1;
  bool wtx = false;
  for (int i = 0; i < count; ++i) {
    bt = std::min(bt, tiled_batch_per_thread(storage, batch[i]));
    const int Q = plans[i]->Q;
    qn = std::max(qn, Q == 1 ? 1 : Q <= 4 ? 4 : Q <= 8 ? 8 : 16);
    wtx |= plans[i]->w_tx != nullptr;
  }
  BatchedArgs a{};
  a.count = count;
  a.first[0] = 0;
  for (int i = 0; i < count; ++i) {
    const das_plan_s* p = plans[i];
    PlanWork& w = a.p[i];
    w.g = call_geom(p, ws[i], batch[i]);
    w.ts = tile_shape(p->tile);
    w.win = make_window(p, w.ts);
    w.ws = ws[i];
    w.x = x[i];
    w.B = batch[i];
    w.ntx = (w.g.n[0] + w.ts.tx - 1) / w.ts.tx;
    w.nty = (w.g.n[1] + w.ts.ty - 1) / w.ts.ty;
    const int ntz = (w.g.n[2] + w.ts.tz - 1) / w.ts.tz;
    w.ntiles = w.ntx * w.nty * ntz;
    a.first[i + 1] = a.first[i] + w.ntiles * ((batch[i] + bt - 1) / bt);
  }
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, plans[0]->device);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (storage == DAS_STORE_F32) e = tiled_batched_f32(a, bt, qn, wtx, cus, st);
  else if (storage == DAS_STORE_F16) e = tiled_batched_f16(a, bt, qn, wtx, cus, st);
  else if (storage == DAS_STORE_FP8_E4M3) e = tiled_batched_fp8(a, bt, qn, wtx, cus, st);
  else e = tiled_batched_bf16(a, bt, qn, wtx, cus, st);
  if (e != hipSuccess) return hip_fail(e, "das_forward_batched launch");
  return DAS_OK;
}

// MFMA plans: time each MFMA launch form on a zeroed workspace of `batch`
// items (the time does not depend on the sample values) and keep the fastest.
static das_status autotune_mfma(das_plan p, int32_t batch, hipStream_t st) {
  const size_t wsb = ws_bytes(p, batch);
  void* ws = nullptr;
  float* x = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&ws, wsb);
  if (e == hipSuccess) e = hipMalloc((void**)&x, sizeof(float) * (size_t)batch * p->N);
  if (e == hipSuccess) e = hipMemsetAsync(ws, 0, wsb, st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int saved = p->mfma_form;
  int best = -1;
  float best_ms = 1e30f;
  das_status ds = DAS_OK;
  const int forms[5] = {DAS_MFMA_COLUMN, DAS_MFMA_SLAB, DAS_MFMA_PERSISTENT, DAS_MFMA_COLUMN_FP8,
                        DAS_MFMA_SLAB_FP8};
  const int nforms = p->cfg.storage == DAS_STORE_FP8_E4M3 ? 5 : 3;
  for (int fi = 0; fi < nforms && e == hipSuccess && ds == DAS_OK; ++fi) {
    p->mfma_form = forms[fi];
    ds = das_forward(p, ws, batch, x, st);  // warm-up
    if (ds == DAS_OK) e = hipEventRecord(e0, st);
    for (int r = 0; r < 2 && e == hipSuccess && ds == DAS_OK; ++r) ds = das_forward(p, ws, batch, x, st);
    if (ds == DAS_OK && e == hipSuccess) e = hipEventRecord(e1, st);
    if (ds == DAS_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (ds == DAS_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (ds == DAS_OK && e == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = forms[fi];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (ws) (void)hipFree(ws);
  if (x) (void)hipFree(x);
  p->mfma_form = best >= 0 ? best : saved;
  if (e != hipSuccess) return hip_fail(e, "das_autotune");
  return ds;
}

das_status das_autotune(das_plan p, int32_t batch, void* stream) {
  if (das_status s = check_plan(p)) return s;
  if (das_status s = check_batch(p, batch)) return s;
  if (p->iq && batch % 2) return fail(DAS_ERR_INVALID_ARG, "complex baseband needs an even batch");
  DeviceGuard dg(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (choose_algo(p, batch) == DAS_ALGO_MFMA) return autotune_mfma(p, batch, st);
  const int saved_algo = p->algo;
  p->algo = DAS_ALGO_TILED;
  const size_t wsb = ws_bytes(p, batch);
  void* ws = nullptr;
  float* x = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&ws, wsb);
  if (e == hipSuccess) e = hipMalloc((void**)&x, sizeof(float) * (size_t)batch * p->N);
  if (e == hipSuccess) e = hipMemsetAsync(ws, 0, wsb, st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int best = -1;
  float best_ms = 1e30f;
  const Geom g = call_geom(p, ws, batch);  // zeroed workspace: FP8 items unscaled
  for (int ti = 0; ti < kNumTiles && e == hipSuccess; ++ti) {
    if (!tiled_fits(p, ti, batch)) continue;
    e = launch_windowed(p, g, ti, ws, batch, x, st);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_windowed(p, g, ti, ws, batch, x, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = ti;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (ws) (void)hipFree(ws);
  if (x) (void)hipFree(x);
  p->algo = saved_algo;
  if (e != hipSuccess) return hip_fail(e, "das_autotune");
  if (best < 0) return fail(DAS_ERR_UNSUPPORTED, "no tile shape fits this geometry");
  p->tile = best;
  return DAS_OK;
}

das_status das_clutter_workspace_bytes(int32_t T, size_t* bytes) {
  if (!bytes) return fail(DAS_ERR_INVALID_ARG, "bytes is NULL");
  if (T < 1 || T > 512) return fail(DAS_ERR_INVALID_ARG, "T must be in [1, 512]");
  *bytes = clutter_workspace_bytes(T);
  return DAS_OK;
}

static das_status check_clutter_args(const float* x, int32_t T, int64_t N, int32_t k_lo,
                                     int32_t k_hi, const float* sv, const float* power) {
  if (!x || !sv || !power) return fail(DAS_ERR_INVALID_ARG, "x, sv or power is NULL");
  if (T < 1 || T > 512) return fail(DAS_ERR_INVALID_ARG, "T must be in [1, 512]");
  if (N < 1) return fail(DAS_ERR_INVALID_ARG, "N must be >= 1");
  if (k_lo < 0 || k_hi <= k_lo || k_hi > T)
    return fail(DAS_ERR_INVALID_ARG, "need 0 <= k_lo < k_hi <= T");
  if (clutter_basis_size(T, k_lo, k_hi) > 64)
    return fail(DAS_ERR_UNSUPPORTED, "at most 64 components may be kept or removed");
  return DAS_OK;
}

static das_status run_clutter(const float* x, int32_t T, int64_t N, int32_t k_lo, int32_t k_hi,
                              float* sv, float* power, float* xf, void* ws, void* stream,
                              const char* where) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = launch_clutter_filter(x, T, N, k_lo, k_hi, sv, power, xf, ws, cus,
                            static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, where);
  return DAS_OK;
}

das_status das_clutter_filter(const float* x, int32_t T, int64_t N, int32_t k_lo, int32_t k_hi,
                              float* sv, float* power, float* xf, void* ws, void* stream) {
  if (das_status s = check_clutter_args(x, T, N, k_lo, k_hi, sv, power)) return s;
  if (!ws) return fail(DAS_ERR_INVALID_ARG, "ws is NULL");
  return run_clutter(x, T, N, k_lo, k_hi, sv, power, xf, ws, stream, "das_clutter_filter launch");
}

das_status das_clutter_filter_noalloc(const float* x, int32_t T, int64_t N, int32_t k_lo,
                                      int32_t k_hi, float* sv, float* power, float* xf,
                                      void* stream) {
  if (das_status s = check_clutter_args(x, T, N, k_lo, k_hi, sv, power)) return s;
  if (T > clutter_static_max_frames())
    return fail(DAS_ERR_INVALID_ARG, "das_clutter_filter_noalloc: T exceeds the static workspace (256 frames)");
  void* ws = nullptr;
  size_t bytes = 0;
  hipError_t e = clutter_static_scratch(&ws, &bytes);
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (static clutter workspace)");
  if (clutter_workspace_bytes(T) > bytes)
    return fail(DAS_ERR_INVALID_ARG, "das_clutter_filter_noalloc: workspace exceeds the static buffer");
  return run_clutter(x, T, N, k_lo, k_hi, sv, power, xf, ws, stream,
                     "das_clutter_filter_noalloc launch");
}

das_status das_debug_delays(das_plan p, int32_t q, int32_t m0, int32_t m1, int32_t n0, int32_t n1,
                            double* f_out, void* stream) {
  if (das_status s = check_plan(p)) return s;
  if (!f_out) return fail(DAS_ERR_INVALID_ARG, "f_out is NULL");
  if (q < 0 || q >= p->Q || m0 < 0 || m1 > p->M || m0 >= m1 || n0 < 0 || n1 > p->N || n0 >= n1)
    return fail(DAS_ERR_INVALID_ARG, "bad q / element / voxel range");
  DeviceGuard dg(p->device);
  hipError_t e = launch_debug_delays(make_geom(p), tile_shape(p->tile), q, m0, m1, n0, n1, f_out,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "das_debug_delays launch");
  return DAS_OK;
}

}  // extern "C"
