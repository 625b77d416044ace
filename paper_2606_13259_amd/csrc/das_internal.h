// Internal declarations shared by the HIP kernels and the C-ABI layer of the
// delay-and-sum library (gfx950).  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "das.h"

namespace dasmi {

// Device view of a plan's geometry; passed to kernels by value.
struct Geom {
  const double* elem;    // [M][3] element positions (m)
  const float* enorm;    // [M][3] unit element normals, or nullptr (= +z)
  const double* txvec;   // [Q][3] plane-wave direction or virtual source
  const double* txoff;   // [Q] path offsets L_q (m)
  const int* txkind;     // [Q] das_tx_kind
  const float* w_tx;     // [Q][N] transmit weights or nullptr (= 1)
  double o[3];           // grid origin (m)
  double s[3];           // grid spacing (m)
  int n[3];              // grid dims
  int M, Q, K;
  double c;              // sound speed (m/s)
  double fs;             // sampling rate (Hz)
  double fsc;            // fs / c   (samples per metre of path)
  double t0fs;           // t0 * fs  (samples)
  int apod;              // das_apod
  float fourF2;          // 4 F^2 (Hann f-number aperture test)
  const float* amax;     // FP8 workspaces: [batch] largest magnitude per item (fixes
                         // its scale), else nullptr
  int iq;                // complex baseband mode: items (2b, 2b+1) are (I, Q)
  double fcfs;           // IQ: carrier / sampling rate (revolutions per sample)
  double fct0;           // IQ: frac(fc t0) (revolutions)
};

// Voxel tile handled by one workgroup of the windowed kernels.
struct TileShape {
  int tx, ty, tz;        // voxels per tile along x, y, z (tx*ty*tz == 256)
  int lx, lxy;           // log2(tx), log2(tx*ty)
  // The windowed forward splits a tile into four wavefront boxes of 64
  // voxels, as near to cubes as the tile allows (the smallest bounding
  // spheres for the per-wavefront element test):
  int wx, wy, wz;        // voxels per wavefront box along x, y, z
  int wlx, wlxy;         // log2(wx), log2(wx*wy)
  int bx, by;            // wavefront boxes along x, y (bx*by*bz == 4)
  int blx, blxy;         // log2(bx), log2(bx*by)
};

// Window geometry of the windowed kernels for one launch (depends on c).
struct Window {
  int dint;              // offset of the tile reference sample inside a window
  int pairs;             // sample pairs per (transmit, element) window
};

// One plan's share of a persistent batched launch (passed by value).
constexpr int MAX_BATCHED = 16;
struct PlanWork {
  Geom g;
  TileShape ts;
  Window win;
  const void* ws;
  float* x;
  int B, ntx, nty, ntiles;
};
struct BatchedArgs {
  PlanWork p[MAX_BATCHED];
  int first[MAX_BATCHED + 1];  // work-item ranges per plan
  int count;
};
hipError_t tiled_batched_f32(const BatchedArgs& a, int bt, int qn, bool wtx, int cus,
                             hipStream_t st);
hipError_t tiled_batched_f16(const BatchedArgs& a, int bt, int qn, bool wtx, int cus,
                             hipStream_t st);
hipError_t tiled_batched_bf16(const BatchedArgs& a, int bt, int qn, bool wtx, int cus,
                              hipStream_t st);
hipError_t tiled_batched_fp8(const BatchedArgs& a, int bt, int qn, bool wtx, int cus,
                             hipStream_t st);

// ---------------------------------------------------------------------------
// Host-side launchers (each returns the hipError_t of its launch).
// ---------------------------------------------------------------------------
// g.amax: the FP8 scale table of the workspace (FP8 storage only).
hipError_t launch_reorder(const Geom& g, int storage, const float* y, int b0, int nb, int btot,
                          void* ws, hipStream_t st);
// amax[b0 .. b0+nb-1] = largest |y| of each item of y[nb][Q][M][K] (the FP8
// scale table; NaN compares above inf).
hipError_t launch_item_absmax(const Geom& g, const float* y, int b0, int nb, float* amax,
                              hipStream_t st);
hipError_t launch_plain_forward(const Geom& g, const float* y, int B, float* x, hipStream_t st);
hipError_t launch_tiled_forward(const Geom& g, int storage, const TileShape& ts, const Window& w,
                                const void* ws, int B, float* x, hipStream_t st);
size_t adjoint_lds_bytes(const Geom& g, const Window& w);
hipError_t launch_adjoint(const Geom& g, const TileShape& ts, const Window& w, const float* gx,
                          int B, float* gy, hipStream_t st);
hipError_t launch_grad_c(const Geom& g, const float* y, const float* gx, int B, float* dLdc,
                         hipStream_t st);
hipError_t launch_debug_delays(const Geom& g, const TileShape& ts, int q, int m0, int m1, int n0,
                               int n1, double* f_out, hipStream_t st);
// Matrix-core locality form (f16 / bf16 / fp8 storage): chunked batch-inner
// workspace [Bp/TW][Q][M][Kc][TW][8].
int mfma_tiles_per_wave(int B);  // 16-column MFMA tiles per wavefront (1, 2 or 4)
int mfma_stack_tiles(int B);     // 16-column tiles per wavefront of the depth-stacked form (1, 2, 4)
int mfma_tile_width(int B);      // batch items per workspace tile (16 x tiles per wavefront)
int mfma_batch_pad(int B);       // batch rounded up to the tile width
int mfma_chunks(int K);
// One plan's share of a persistent MFMA launch (passed by value).
struct MfmaWork {
  Geom g;
  const void* ws;
  float* x;
  int B, TW, Kc, ngx, ngy, ngroups, nbx;  // ngroups: wavefront columns
  int nb;                                 // 16-column batch tiles per wavefront
};
struct MfmaBatchedArgs {
  MfmaWork p[MAX_BATCHED];
  int first[MAX_BATCHED + 1];  // work-item ranges per plan
  int count;
};
// Fills the derived fields (column counts, work-list ranges) of `a` from
// g, ws, x, B, TW, Kc of each plan and launches the persistent MFMA kernel,
// which schedules its items through the device counters `ctr`
// (mfma_batched_counter_bytes(), zeroed on `st` before the launch).  iq: every
// plan is in complex baseband mode (f16 or FP8 storage).
size_t mfma_batched_counter_bytes();
// Whether a single-plan forward should use the persistent kernel.
bool mfma_prefers_persistent(int storage, int B);
hipError_t launch_mfma_batched(MfmaBatchedArgs& a, unsigned* ctr, int storage, bool iq, int cus,
                               hipStream_t st);
size_t mfma_workspace_elems(const Geom& g, int B);  // samples (1, 2 bytes each)
hipError_t launch_mfma_reorder(const Geom& g, int storage, const float* y, int b0, int nb, int btot,
                               void* ws, hipStream_t st);
// Plain MFMA launch with 4 x 4 x 4 wavefront columns, or 8 x 8 x 1 slabs;
// FP8 storage: fp8_operands contracts the stored codes with FP8 weights on
// the FP8 matrix instructions instead of decoding them to f16.
hipError_t launch_mfma_forward(const Geom& g, int storage, const void* ws, int B, float* x,
                               bool slab, bool fp8_operands, hipStream_t st);
// Complex baseband (IQ) items in (I, Q) column pairs, f16 or FP8 storage.
hipError_t launch_mfma_forward_iq(const Geom& g, int storage, const void* ws, int B, float* x,
                                  bool slab, hipStream_t st);

// Windowed forward, one instantiation set per storage type.
hipError_t tiled_forward_f32(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                             int B, float* x, hipStream_t st);
hipError_t tiled_forward_f16(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                             int B, float* x, hipStream_t st);
hipError_t tiled_forward_bf16(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                              int B, float* x, hipStream_t st);
hipError_t tiled_forward_fp8(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                             int B, float* x, hipStream_t st);
// Complex baseband (IQ pairs), f32 storage.
hipError_t tiled_forward_f32_cubic(const Geom& g, const TileShape& ts, const Window& w,
                                   const void* ws, int B, float* x, hipStream_t st);
hipError_t tiled_forward_f32_iq(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                                int B, float* x, hipStream_t st);
size_t tiled_lds_f32(const Geom& g, int bt, const Window& w);
size_t tiled_lds_f16(const Geom& g, int bt, const Window& w);
size_t tiled_lds_bf16(const Geom& g, int bt, const Window& w);
size_t tiled_lds_fp8(const Geom& g, int bt, const Window& w);

// Rank-truncation clutter filter (k_clutter.hip).
size_t clutter_workspace_bytes(int T);
int clutter_static_max_frames();                              // T limit of the static workspace
hipError_t clutter_static_scratch(void** ptr, size_t* bytes);  // this device's static workspace
int clutter_basis_size(int T, int k_lo, int k_hi);  // components the projection uses
hipError_t launch_clutter_filter(const float* x, int T, long long N, int k_lo, int k_hi, float* sv,
                                 float* pd, float* xf, void* ws, int cus, hipStream_t st);

// LDS bytes the tiled forward kernel needs (0 if it cannot run this shape).
size_t tiled_lds_bytes(const Geom& g, int storage, int bt, const Window& w);
int tiled_batch_per_thread(int storage, int B);

}  // namespace dasmi
