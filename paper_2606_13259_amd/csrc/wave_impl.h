// Wavefront-tiled forward kernel for the VALU (paper, Sec. 3.2 batch-inner
// tiling and Sec. 3.3 mixed-precision storage, re-designed for gfx950).
//
// Each 64-lane wavefront owns a box of 64 neighbouring voxels (one per lane)
// and BT batch items, and runs independently of the other wavefronts of its
// workgroup: no workgroup barrier anywhere.
//
//   * Elements are visited in blocks of 64: lane l tests element m0 + l
//     against the wavefront box's bounding sphere (receive-aperture cone,
//     conservative) and forms its FP64 tile-relative reference terms
//     (das_device.h); a ballot gives the block's active elements, which the
//     wavefront then walks with find-first-set, broadcasting each element's
//     terms with readlane.
//   * For each active element the wavefront stages the QN sample windows of
//     its (transmit, element) channels: lane p loads sample p of every window
//     with a bounds-checked buffer load (the buffer of a channel spans exactly
//     its K samples, so taps outside [0, K) read zero at no cost), converts to
//     FP32 and writes it to a per-wavefront LDS buffer; each voxel lane then
//     reads its two taps with one ds_read2_b32.  The loads of the next active
//     element are issued before the current element is interpolated
//     (register double buffering), so load latency hides behind arithmetic.
//   * The window of channel (q, m) starts at ktx_q + krx_m - dint, where dint
//     bounds |f - (ktx + krx)| over the box (triangle inequality on the box
//     half-diagonal).
//   * Block ids are remapped so that each XCD (and its L2) receives a
//     contiguous range of boxes, whose windows overlap.
//
// Arithmetic: delays are tile-relative FP32 with FP64 reference terms;
// samples are converted to FP32 before interpolation; accumulation is FP32.
// Transmits are processed in groups of QN (compile-time); a group that is not
// full is padded with zero-weight transmits.
#pragma once
#include "das_device.h"

namespace dasmi {
namespace wavek {

constexpr int WAVES = 4;  // wavefronts per workgroup

// Buffer resource over one channel [K * B] of the workspace (bytes = K*B*sizeof(T)).
__device__ inline __amdgpu_buffer_rsrc_t channel_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <class T, int BT> __device__ inline void load_taps(__amdgpu_buffer_rsrc_t r, int off, float* v);
template <> __device__ inline void load_taps<float, 1>(__amdgpu_buffer_rsrc_t r, int off, float* v) {
  v[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ inline void load_taps<float, 2>(__amdgpu_buffer_rsrc_t r, int off, float* v) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  const u2 d = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  v[0] = __uint_as_float(d.x);
  v[1] = __uint_as_float(d.y);
}
template <> __device__ inline void load_taps<float, 4>(__amdgpu_buffer_rsrc_t r, int off, float* v) {
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  const u4 d = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  v[0] = __uint_as_float(d.x);
  v[1] = __uint_as_float(d.y);
  v[2] = __uint_as_float(d.z);
  v[3] = __uint_as_float(d.w);
}
__device__ inline float h2f(uint32_t bits16) {
  _Float16 h = __builtin_bit_cast(_Float16, (uint16_t)bits16);
  return (float)h;
}
template <> __device__ inline void load_taps<_Float16, 1>(__amdgpu_buffer_rsrc_t r, int off, float* v) {
  v[0] = h2f(__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
}
template <> __device__ inline void load_taps<_Float16, 2>(__amdgpu_buffer_rsrc_t r, int off, float* v) {
  const uint32_t d = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  v[0] = h2f(d & 0xffffu);
  v[1] = h2f(d >> 16);
}
template <> __device__ inline void load_taps<_Float16, 4>(__amdgpu_buffer_rsrc_t r, int off, float* v) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  const u2 d = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  v[0] = h2f(d.x & 0xffffu);
  v[1] = h2f(d.x >> 16);
  v[2] = h2f(d.y & 0xffffu);
  v[3] = h2f(d.y >> 16);
}
template <> __device__ inline void load_taps<uint16_t, 1>(__amdgpu_buffer_rsrc_t r, int off, float* v) {
  v[0] = __uint_as_float(((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0)) << 16);
}
template <> __device__ inline void load_taps<uint16_t, 2>(__amdgpu_buffer_rsrc_t r, int off, float* v) {
  const uint32_t d = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  v[0] = __uint_as_float(d << 16);
  v[1] = __uint_as_float(d & 0xffff0000u);
}
template <> __device__ inline void load_taps<uint16_t, 4>(__amdgpu_buffer_rsrc_t r, int off, float* v) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  const u2 d = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  v[0] = __uint_as_float(d.x << 16);
  v[1] = __uint_as_float(d.x & 0xffff0000u);
  v[2] = __uint_as_float(d.y << 16);
  v[3] = __uint_as_float(d.y & 0xffff0000u);
}

// Conservative sphere-cone test (see tiled_impl.h for the derivation).
__device__ inline bool sphere_in_cone(float ex, float ey, float ez, float nx, float ny, float nz,
                                      float R, float cth, float sth) {
  const float D2 = ex * ex + ey * ey + ez * ez;
  if (D2 <= R * R * 1.0001f + 1e-18f) return true;
  const float invD = __builtin_amdgcn_rsqf(D2);
  const float cphi = (ex * nx + ey * ny + ez * nz) * invD;
  const float sb = R * invD;
  const float cb = __builtin_amdgcn_sqrtf(fmaxf(0.f, 1.f - sb * sb));
  return cphi > cth * cb - sth * sb - 1e-4f;
}

// Box of 64 voxels owned by one wavefront.
struct BoxShape {
  int bx, by, bz;   // bx*by*bz == 64, powers of two
  int lx, lxy;      // log2(bx), log2(bx*by)
};

template <class T, int BT, int QN, bool WTX>
__global__ __launch_bounds__(64 * WAVES) void wave_forward(Geom g, BoxShape bs, Window win,
                                                          const T* __restrict__ ws, int B,
                                                          float* __restrict__ x, int nbx, int nby,
                                                          int nboxes, int per_xcd) {
  extern __shared__ __align__(16) float lds[];
  const int W = win.pairs + 1;  // samples per window, <= 64
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // One window buffer per wavefront: LDS operations of a wavefront execute in
  // issue order, so the staging writes of element j+1 cannot overtake the
  // tap reads of element j.
  float* buf = lds + wave * QN * W * BT;

  const int blk = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  const int box = blk * WAVES + wave;
  if (box >= nboxes) return;  // whole wavefront
  const int bxi = box % nbx, byi = (box / nbx) % nby, bzi = box / (nbx * nby);
  const int lx = lane & (bs.bx - 1), ly = (lane >> bs.lx) & (bs.by - 1), lz = lane >> bs.lxy;
  const int ix = bxi * bs.bx + lx, iy = byi * bs.by + ly, iz = bzi * bs.bz + lz;
  const int b0 = blockIdx.y * BT;
  const int K = g.K, M = g.M;
  const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];

  const float hx = 0.5f * (bs.bx - 1), hy = 0.5f * (bs.by - 1), hz = 0.5f * (bs.bz - 1);
  double px, py, pz;
  tile_ref_point(g, bxi * bs.bx + (double)hx, byi * bs.by + (double)hy, bzi * bs.bz + (double)hz,
                 px, py, pz);
  const float sx = (float)g.s[0], sy = (float)g.s[1], sz = (float)g.s[2];
  const float dx = ((float)lx - hx) * sx, dy = ((float)ly - hy) * sy, dz = ((float)lz - hz) * sz;
  const float dp2 = dx * dx + dy * dy + dz * dz;
  const float fscf = (float)g.fsc;
  const bool inside = in_grid(g, ix, iy, iz);
  const int n = grid_index(g, ix, iy, iz);
  const float Rbox = sqrtf(hx * hx * sx * sx + hy * hy * sy * sy + hz * hz * sz * sz);
  const bool hann = g.apod == DAS_APOD_HANN_FNUM;
  const float cth = hann ? sqrtf(g.fourF2) * rsqrtf(1.f + g.fourF2) : -1.f;
  const float sth = hann ? rsqrtf(1.f + g.fourF2) : 0.f;
  const uint32_t chan_bytes = (uint32_t)((size_t)K * B * sizeof(T));
  const size_t chan_elems = (size_t)K * B;

  float acc[BT];
#pragma unroll
  for (int b = 0; b < BT; ++b) acc[b] = 0.f;

  for (int q0 = 0; q0 < g.Q; q0 += QN) {
    const int qn = min(QN, g.Q - q0);
    // transmit terms: lane q forms those of transmit q0 + q
    TxRef mine = {};
    if (lane < qn) mine = make_tx_ref(g, q0 + lane, px, py, pz);
    float bq[QN], wq[WTX ? QN : 1];
    int soff[QN];  // per-lane staging offset (elements) of window q, without krx
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      TxRef r;
      r.kind = __shfl(mine.kind, q);
      r.vx = __shfl(mine.vx, q);
      r.vy = __shfl(mine.vy, q);
      r.vz = __shfl(mine.vz, q);
      r.vn = __shfl(mine.vn, q);
      const float gq = __shfl(mine.g, q);
      const int kq = __shfl(mine.ktx, q);
      bq[q] = q < qn ? fmaf(delta_tx(r, dx, dy, dz, dp2), fscf, gq) : 0.f;
      if (WTX) wq[WTX ? q : 0] = (q < qn && inside) ? g.w_tx[(size_t)(q0 + q) * N + n] : 0.f;
      soff[q] = kq - win.dint + lane;
    }

    for (int m0 = 0; m0 < M; m0 += 64) {
      // lane l: element m0 + l -> aperture test + FP64 reference terms
      const int me = m0 + lane;
      bool on = false;
      float rex = 0.f, rey = 0.f, rez = 0.f, rh = 0.f;
      int rk = 0;
      if (me < M) {
        const double ex = px - g.elem[3 * me + 0];
        const double ey = py - g.elem[3 * me + 1];
        const double ez = pz - g.elem[3 * me + 2];
        rex = (float)ex;
        rey = (float)ey;
        rez = (float)ez;
        on = true;
        if (hann) {
          float nx = 0.f, ny = 0.f, nz = 1.f;
          if (g.enorm) {
            nx = g.enorm[3 * me + 0];
            ny = g.enorm[3 * me + 1];
            nz = g.enorm[3 * me + 2];
          }
          on = sphere_in_cone(rex, rey, rez, nx, ny, nz, Rbox, cth, sth);
        }
        if (on) {
          const double R = sqrt(ex * ex + ey * ey + ez * ez);
          const double fr = R * g.fsc;
          const double fl = floor(fr);
          rh = (float)(fr - fl);
          rk = (int)fl;
        }
      }
      uint64_t amask = __ballot(on);
      if (amask == 0ull) continue;

      float nxt[QN][BT];
      auto issue = [&](int j) {
        const int m = m0 + j;
        const int krx = __builtin_amdgcn_readlane(rk, j);
#pragma unroll
        for (int q = 0; q < QN; ++q) {
          const T* chan = ws + ((size_t)(q0 + q) * M + m) * chan_elems + b0;
          const __amdgpu_buffer_rsrc_t rs = channel_rsrc(chan, q < qn && lane < W ? chan_bytes : 0u);
          load_taps<T, BT>(rs, (soff[q] + krx) * B * (int)sizeof(T), nxt[q]);
        }
      };
      int j = __builtin_ctzll(amask);
      amask &= amask - 1ull;
      issue(j);
      while (true) {
        float* cur = buf;
        // stage the loaded windows of element j
#pragma unroll
        for (int q = 0; q < QN; ++q)
          if (lane < W) {
#pragma unroll
            for (int b = 0; b < BT; ++b) cur[(q * W + lane) * BT + b] = nxt[q][b];
          }
        const int jcur = j;
        const bool more = amask != 0ull;
        if (more) {
          j = __builtin_ctzll(amask);
          amask &= amask - 1ull;
          issue(j);  // prefetch the next active element
        }
        // interpolate and accumulate element jcur
        const float ex = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rex), jcur));
        const float ey = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rey), jcur));
        const float ez = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rez), jcur));
        const float h = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rh), jcur));
        const float w = rx_weight(g, m0 + jcur, ex + dx, ey + dy, ez + dz);
        const float en = __builtin_amdgcn_sqrtf(ex * ex + ey * ey + ez * ez);
        const float a = fmaf(delta_dist(ex, ey, ez, en, dx, dy, dz, dp2), fscf, h);
        const float* base = cur + win.dint * BT;
        constexpr int QR = QN * BT <= 8 ? QN : (8 / BT < 1 ? 1 : 8 / BT);
#pragma unroll
        for (int qa = 0; qa < QN; qa += QR) {
          float s1[QR][BT], s2[QR][BT], al[QR];
#pragma unroll
          for (int r = 0; r < QR; ++r) {
            const float f = a + bq[qa + r];
            const float fl = floorf(f);
            al[r] = f - fl;
            const float* pp = base + ((qa + r) * W + (int)fl) * BT;
#pragma unroll
            for (int b = 0; b < BT; ++b) {
              s1[r][b] = pp[b];
              s2[r][b] = pp[BT + b];
            }
          }
#pragma unroll
          for (int r = 0; r < QR; ++r) {
            const float wt = WTX ? w * wq[WTX ? qa + r : 0] : w;
#pragma unroll
            for (int b = 0; b < BT; ++b)
              acc[b] = fmaf(wt, fmaf(al[r], s2[r][b], fmaf(-al[r], s1[r][b], s1[r][b])), acc[b]);
          }
        }
        if (!more) break;
      }
    }
  }
  if (inside) {
#pragma unroll
    for (int b = 0; b < BT; ++b)
      if (b0 + b < B) x[(size_t)(b0 + b) * N + n] = acc[b];
  }
}

inline size_t lds_bytes(int QN, int BT, const Window& w) {
  return (size_t)WAVES * QN * (w.pairs + 1) * BT * 4;
}

template <class T, int BT, int QN, bool WTX>
hipError_t launch_t(const Geom& g, const BoxShape& bs, const Window& w, const void* ws, int B,
                    float* x, hipStream_t st) {
  const int nbx = (g.n[0] + bs.bx - 1) / bs.bx, nby = (g.n[1] + bs.by - 1) / bs.by,
            nbz = (g.n[2] + bs.bz - 1) / bs.bz;
  const int nboxes = nbx * nby * nbz;
  const int nblk = (nboxes + WAVES - 1) / WAVES;
  const int per_xcd = (nblk + 7) / 8;
  const size_t lds = lds_bytes(QN, BT, w);
  auto kern = wave_forward<T, BT, QN, WTX>;
  if (lds > 65536) {
    hipError_t e =
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(per_xcd * 8, (B + BT - 1) / BT), dim3(64 * WAVES), lds, st, g, bs, w,
                     static_cast<const T*>(ws), B, x, nbx, nby, nboxes, per_xcd);
  return hipGetLastError();
}

inline int group_size(int Q) { return Q == 1 ? 1 : Q <= 4 ? 4 : Q <= 8 ? 8 : 16; }

template <class T, int BT>
hipError_t launch_bt(const Geom& g, const BoxShape& bs, const Window& w, const void* ws, int B,
                     float* x, hipStream_t st) {
  const bool wtx = g.w_tx != nullptr;
  switch (group_size(g.Q)) {
    case 1: return wtx ? launch_t<T, BT, 1, true>(g, bs, w, ws, B, x, st)
                       : launch_t<T, BT, 1, false>(g, bs, w, ws, B, x, st);
    case 4: return wtx ? launch_t<T, BT, 4, true>(g, bs, w, ws, B, x, st)
                       : launch_t<T, BT, 4, false>(g, bs, w, ws, B, x, st);
    case 8: return wtx ? launch_t<T, BT, 8, true>(g, bs, w, ws, B, x, st)
                       : launch_t<T, BT, 8, false>(g, bs, w, ws, B, x, st);
    default: return wtx ? launch_t<T, BT, 16, true>(g, bs, w, ws, B, x, st)
                        : launch_t<T, BT, 16, false>(g, bs, w, ws, B, x, st);
  }
}

template <class T>
hipError_t launch(const Geom& g, const BoxShape& bs, const Window& w, const void* ws, int B,
                  float* x, hipStream_t st) {
  if (B >= 4) return launch_bt<T, 4>(g, bs, w, ws, B, x, st);
  if (B >= 2) return launch_bt<T, 2>(g, bs, w, ws, B, x, st);
  return launch_bt<T, 1>(g, bs, w, ws, B, x, st);
}

}  // namespace wavek
}  // namespace dasmi
