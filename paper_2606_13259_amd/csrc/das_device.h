// Device-side building blocks of delay formation (paper, Sec. 2, Eq. (1) and
// its footnote) shared by the forward, adjoint, gradient and debug kernels.
//
// Delay formation is tile-relative.  For a voxel tile with reference point p0
// (the tile centre) and a voxel p = p0 + dp:
//   * per (tile, element m), in FP64: R0 = |p0 - r_m|; R0*fs/c is split into
//     an integer krx and a fraction H in [0, 1);
//   * per (tile, transmit q), in FP64: T0 = D_tx(p0); T0*fs/c - t0*fs is split
//     into ktx and a fraction G in [0, 1);
//   * per voxel, in FP32: the path differences |p - r| - |p0 - r| and
//     D_tx(p) - D_tx(p0), each in a cancellation-free form, scaled by fs/c;
//   * f = (ktx + krx) + (A + Bq) with A = H + drx*fs/c and Bq = G + dtx*fs/c.
// |dp| is at most half the tile diagonal, so every FP32 quantity stays small
// (tens of samples) and the index error stays near 1e-6 samples, where the
// naive FP32 form |p - r| / c * fs loses ~1e-4 samples at k ~ 1000.
#pragma once

#include "das_internal.h"

namespace dasmi {

// Per-element FP32 view relative to a tile reference.
struct RxRef {
  float ex, ey, ez;  // p0 - r_m
  float en;          // |p0 - r_m|
  float h;           // frac(R0 * fs / c)
  int krx;           // floor(R0 * fs / c)
};

// Per-transmit FP32 view relative to a tile reference.
struct TxRef {
  float vx, vy, vz;  // PLANE: u; DIVERGING: p0 - v
  float vn;          // DIVERGING: |p0 - v|
  float g;           // frac(D_tx(p0) * fs / c - t0 fs)
  int ktx;           // floor(...)
  int kind;
};

__device__ inline void tile_ref_point(const Geom& g, double cx, double cy, double cz, double& px,
                                      double& py, double& pz) {
  px = g.o[0] + cx * g.s[0];
  py = g.o[1] + cy * g.s[1];
  pz = g.o[2] + cz * g.s[2];
}

__device__ inline RxRef make_rx_ref(const Geom& g, int m, double px, double py, double pz) {
  RxRef r;
  const double ex = px - g.elem[3 * m + 0];
  const double ey = py - g.elem[3 * m + 1];
  const double ez = pz - g.elem[3 * m + 2];
  const double R = sqrt(ex * ex + ey * ey + ez * ez);
  const double fr = R * g.fsc;
  const double fl = floor(fr);
  r.ex = (float)ex;
  r.ey = (float)ey;
  r.ez = (float)ez;
  r.en = (float)R;
  r.h = (float)(fr - fl);
  r.krx = (int)fl;
  return r;
}

__device__ inline TxRef make_tx_ref(const Geom& g, int q, double px, double py, double pz) {
  TxRef t;
  const int kind = g.txkind[q];
  const double vx = g.txvec[3 * q + 0], vy = g.txvec[3 * q + 1], vz = g.txvec[3 * q + 2];
  double d;
  t.kind = kind;
  t.vn = 0.f;
  if (kind == DAS_TX_PLANE) {
    d = vx * px + vy * py + vz * pz;
    t.vx = (float)vx;
    t.vy = (float)vy;
    t.vz = (float)vz;
  } else if (kind == DAS_TX_DIVERGING) {
    const double ax = px - vx, ay = py - vy, az = pz - vz;
    d = sqrt(ax * ax + ay * ay + az * az);
    t.vx = (float)ax;
    t.vy = (float)ay;
    t.vz = (float)az;
    t.vn = (float)d;
  } else {
    d = 0.0;
    t.vx = t.vy = t.vz = 0.f;
  }
  const double ft = (d - g.txoff[q]) * g.fsc - g.t0fs;
  const double fl = floor(ft);
  t.g = (float)(ft - fl);
  t.ktx = (int)fl;
  return t;
}

// |e + dp| - |e| without cancellation: (2 e.dp + dp.dp) / (|e + dp| + |e|).
// dp2 = dp.dp is passed in (constant per voxel).
__device__ inline float delta_dist(float ex, float ey, float ez, float en, float dx, float dy,
                                   float dz, float dp2) {
  const float ax = ex + dx, ay = ey + dy, az = ez + dz;
  const float r2 = ax * ax + ay * ay + az * az;
  const float num = 2.f * (ex * dx + ey * dy + ez * dz) + dp2;
  return num * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(r2) + en);
}

// Transmit path difference D_tx(p0 + dp) - D_tx(p0), FP32.
__device__ inline float delta_tx(const TxRef& t, float dx, float dy, float dz, float dp2) {
  if (t.kind == DAS_TX_PLANE) return t.vx * dx + t.vy * dy + t.vz * dz;
  if (t.kind == DAS_TX_DIVERGING) return delta_dist(t.vx, t.vy, t.vz, t.vn, dx, dy, dz, dp2);
  return 0.f;
}

// Receive weight (Hann with f-number F, or uniform) for d = p - r_m and unit
// normal (nx, ny, nz):  z = d.n, rho = |d - z n|, a = z / (2F);
// w = (1 + cos(pi rho / a)) / 2 = cos^2(pi rho / (2a)) inside the cone.
// cos(pi sqrt(t) / 2) for t = rho^2/a^2 in [0, 1) is evaluated as its Taylor
// series in t (entire in t, no square root), 8 terms: error < 1e-10.
// The weight from the axial distance z and the squared lateral distance rho2.
__device__ inline float hann_weight(float z, float rho2, float fourF2) {
  const float zz = z * z;
  const float t4 = rho2 * fourF2;
  if (!(z > 0.f) || !(t4 < zz)) return 0.f;
  const float t = t4 * __builtin_amdgcn_rcpf(zz);
  const float u = -2.4674011002723395f * t;  // -(pi^2 / 4) t
  float c = 1.1470745597729725e-11f;          // 1/14!
  c = fmaf(c, u, 2.08767569878681e-09f);      // 1/12!
  c = fmaf(c, u, 2.755731922398589e-07f);     // 1/10!
  c = fmaf(c, u, 2.48015873015873e-05f);      // 1/8!
  c = fmaf(c, u, 1.388888888888889e-03f);     // 1/6!
  c = fmaf(c, u, 4.1666666666666664e-02f);    // 1/4!
  c = fmaf(c, u, 0.5f);                       // 1/2!
  c = fmaf(c, u, 1.0f);
  return c * c;
}

__device__ inline float hann_fnum(float dx, float dy, float dz, float nx, float ny, float nz,
                                  float fourF2) {
  const float z = dx * nx + dy * ny + dz * nz;
  const float lx = dx - z * nx, ly = dy - z * ny, lz = dz - z * nz;
  return hann_weight(z, lx * lx + ly * ly + lz * lz, fourF2);
}

__device__ inline float rx_weight(const Geom& g, int m, float dx, float dy, float dz) {
  if (g.apod != DAS_APOD_HANN_FNUM) return 1.f;
  // default normals (+z): z = dz and rho^2 = dx^2 + dy^2 directly
  if (!g.enorm) return hann_weight(dz, dx * dx + dy * dy, g.fourF2);
  return hann_fnum(dx, dy, dz, g.enorm[3 * m + 0], g.enorm[3 * m + 1], g.enorm[3 * m + 2],
                   g.fourF2);
}

// Is any point of the sphere (centre c, radius R) inside the receive cone of
// element m (apex r_m, axis n_m, half-angle atan(1/(2F)))?  Conservative.
__device__ inline bool cone_hits_sphere(const Geom& g, int m, double cx, double cy, double cz,
                                        float R, float tan_half) {
  const float ex = (float)(cx - g.elem[3 * m + 0]);
  const float ey = (float)(cy - g.elem[3 * m + 1]);
  const float ez = (float)(cz - g.elem[3 * m + 2]);
  const float D = sqrtf(ex * ex + ey * ey + ez * ez);
  if (D <= R * 1.001f) return true;
  float nx = 0.f, ny = 0.f, nz = 1.f;
  if (g.enorm) {
    nx = g.enorm[3 * m + 0];
    ny = g.enorm[3 * m + 1];
    nz = g.enorm[3 * m + 2];
  }
  const float z = ex * nx + ey * ny + ez * nz;
  const float lx = ex - z * nx, ly = ey - z * ny, lz = ez - z * nz;
  const float rho = sqrtf(lx * lx + ly * ly + lz * lz);
  const float phi = atan2f(rho, z);
  const float beta = asinf(fminf(1.f, R / D));
  return phi < atanf(tan_half) + beta + 1e-3f;
}

// Compact into act[] (ascending) the elements whose receive cone can reach a
// tile with reference point p and half extents (hx, hy, hz) voxels; returns
// their number.  All 256 threads of the block must call it.  wcount: 4 ints
// of LDS scratch.  Uniform apodization keeps every element.
__device__ inline int cull_elements(const Geom& g, double px, double py, double pz, float hx,
                                    float hy, float hz, int* wcount, uint16_t* act) {
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const float R = sqrtf(hx * hx * (float)(g.s[0] * g.s[0]) + hy * hy * (float)(g.s[1] * g.s[1]) +
                        hz * hz * (float)(g.s[2] * g.s[2]));
  const bool hann = g.apod == DAS_APOD_HANN_FNUM;
  const float tan_half = hann ? 0.5f * sqrtf(4.f / g.fourF2) : 0.f;
  int nact = 0;
  for (int base = 0; base < g.M; base += 256) {
    const int m = base + t;
    bool on = m < g.M;
    if (on && hann) on = cone_hits_sphere(g, m, px, py, pz, R, tan_half);
    const uint64_t mask = __ballot(on);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wave] = __popcll(mask);
    __syncthreads();
    int off = nact;
    for (int w = 0; w < wave; ++w) off += wcount[w];
    if (on) act[off + before] = (uint16_t)m;
    nact += wcount[0] + wcount[1] + wcount[2] + wcount[3];
    __syncthreads();
  }
  return nact;
}

// floor(x) as an integer in one VALU instruction (v_cvt_flr_i32_f32), and the
// matching fraction x - floor(x) (v_fract_f32).
__device__ inline int floor_i32(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}
__device__ inline float frac_f32(float x) { return __builtin_amdgcn_fractf(x); }

// Voxel-grid helpers.
__device__ inline int grid_index(const Geom& g, int ix, int iy, int iz) {
  return ix + g.n[0] * (iy + g.n[1] * iz);
}
__device__ inline bool in_grid(const Geom& g, int ix, int iy, int iz) {
  return ix < g.n[0] && iy < g.n[1] && iz < g.n[2];
}

// Storage conversions (round to nearest even).
__device__ inline float load_f(const float* p) { return *p; }
__device__ inline float load_f(const _Float16* p) { return (float)(*p); }
__device__ inline float load_f(const uint16_t* p) {  // bf16 bits
  return __uint_as_float(((uint32_t)(*p)) << 16);
}

}  // namespace dasmi
