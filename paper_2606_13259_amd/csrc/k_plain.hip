// Plain forward kernel: the per-voxel mapping of the paper's baseline
// (Sec. 3.1, Alg. 1) written for 64-lane wavefronts.
//
// One lane per voxel; each wavefront owns a 4x4x4 voxel block, which is also
// the reference tile of the tile-relative delay formation (das_device.h).
// Each lane handles BT consecutive batch items, reusing the delays and weights
// across them.  Samples are gathered straight from the caller's layout
// y[B][Q][M][K] f32 (no reorder), with per-tap zero padding.
// Loop order: elements outer, transmits inner, so the receive geometry of a
// (voxel, element) pair is formed once and reused for all Q transmits.  The
// FP64 per-(tile, element) reference terms are formed by lane (m mod 64) and
// broadcast with readlane.
#include "das_device.h"

namespace dasmi {
namespace {

constexpr int QG = 16;  // transmits held in registers per pass

template <int BT>
__global__ __launch_bounds__(256) void plain_forward(Geom g, const float* __restrict__ y, int B,
                                                     float* __restrict__ x, int nbx, int nby,
                                                     int nblocks) {
  const int lane = threadIdx.x & 63;
  const int blk = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blk >= nblocks) return;
  const int bxi = blk % nbx, byi = (blk / nbx) % nby, bzi = blk / (nbx * nby);
  const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
  const int ix = bxi * 4 + lx, iy = byi * 4 + ly, iz = bzi * 4 + lz;
  const int b0 = blockIdx.y * BT;

  double px, py, pz;
  tile_ref_point(g, bxi * 4 + 1.5, byi * 4 + 1.5, bzi * 4 + 1.5, px, py, pz);
  const float dx = (float)(lx - 1.5f) * (float)g.s[0];
  const float dy = (float)(ly - 1.5f) * (float)g.s[1];
  const float dz = (float)(lz - 1.5f) * (float)g.s[2];
  const float dp2 = dx * dx + dy * dy + dz * dz;
  const float fscf = (float)g.fsc;
  const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
  const int n = grid_index(g, ix, iy, iz);
  const bool inside = in_grid(g, ix, iy, iz);
  const size_t MK = (size_t)g.M * g.K;
  const size_t QMK = (size_t)g.Q * MK;

  float acc[BT];
#pragma unroll
  for (int b = 0; b < BT; ++b) acc[b] = 0.f;

  for (int q0 = 0; q0 < g.Q; q0 += QG) {
    const int qn = min(QG, g.Q - q0);
    // transmit terms of this lane's voxel
    float bq[QG], wq[QG];
    int ktx[QG];
    {
      TxRef mine = {};
      if (lane < qn) mine = make_tx_ref(g, q0 + lane, px, py, pz);
#pragma unroll
      for (int q = 0; q < QG; ++q) {
        if (q < qn) {
          TxRef t;
          t.kind = g.txkind[q0 + q];
          t.vx = __shfl(mine.vx, q);
          t.vy = __shfl(mine.vy, q);
          t.vz = __shfl(mine.vz, q);
          t.vn = __shfl(mine.vn, q);
          const float gq = __shfl(mine.g, q);
          ktx[q] = __shfl(mine.ktx, q);
          bq[q] = fmaf(delta_tx(t, dx, dy, dz, dp2), fscf, gq);
          wq[q] = (g.w_tx && inside) ? g.w_tx[(size_t)(q0 + q) * N + n] : 1.f;
        } else {
          bq[q] = 0.f;
          ktx[q] = 0;
          wq[q] = 0.f;
        }
      }
    }
    for (int m0 = 0; m0 < g.M; m0 += 64) {
      RxRef mine = {};
      if (m0 + lane < g.M) mine = make_rx_ref(g, m0 + lane, px, py, pz);
      const int mn = min(64, g.M - m0);
      for (int mm = 0; mm < mn; ++mm) {
        const int m = m0 + mm;
        const float ex_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.ex), mm));
        const float ey_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.ey), mm));
        const float ez_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.ez), mm));
        const float en_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.en), mm));
        const float h_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.h), mm));
        const int krx = __builtin_amdgcn_readlane(mine.krx, mm);
        const float ax = ex_ + dx, ay = ey_ + dy, az = ez_ + dz;
        const float w = rx_weight(g, m, ax, ay, az);
        const float a = fmaf(delta_dist(ex_, ey_, ez_, en_, dx, dy, dz, dp2), fscf, h_);
        const float* ym = y + (size_t)m * g.K;
#pragma unroll
        for (int q = 0; q < QG; ++q) {
          if (q < qn) {
            const float f = a + bq[q];
            const float fl = floorf(f);
            const float al = f - fl;
            const int k = (int)fl + ktx[q] + krx;
            const float wt = w * wq[q];
            const float* yq = ym + (size_t)(q0 + q) * MK;
#pragma unroll
            for (int b = 0; b < BT; ++b) {
              if (b0 + b < B) {
                const float* yb = yq + (size_t)(b0 + b) * QMK;
                const float s1 = (k >= 0 && k < g.K) ? yb[k] : 0.f;
                const float s2 = (k + 1 >= 0 && k + 1 < g.K) ? yb[k + 1] : 0.f;
                acc[b] = fmaf(wt, fmaf(al, s2 - s1, s1), acc[b]);
              }
            }
          }
        }
      }
    }
  }
  if (inside) {
#pragma unroll
    for (int b = 0; b < BT; ++b)
      if (b0 + b < B) x[(size_t)(b0 + b) * N + n] = acc[b];
  }
}

template <int BT>
hipError_t plain_t(const Geom& g, const float* y, int B, float* x, hipStream_t st) {
  const int nbx = (g.n[0] + 3) / 4, nby = (g.n[1] + 3) / 4, nbz = (g.n[2] + 3) / 4;
  const int nblocks = nbx * nby * nbz;
  dim3 grid((nblocks + 3) / 4, (B + BT - 1) / BT);
  hipLaunchKernelGGL(plain_forward<BT>, grid, dim3(256), 0, st, g, y, B, x, nbx, nby, nblocks);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_plain_forward(const Geom& g, const float* y, int B, float* x, hipStream_t st) {
  if (B >= 8) return plain_t<8>(g, y, B, x, st);
  if (B >= 4) return plain_t<4>(g, y, B, x, st);
  if (B >= 2) return plain_t<2>(g, y, B, x, st);
  return plain_t<1>(g, y, B, x, st);
}

}  // namespace dasmi
