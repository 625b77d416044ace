// Windowed forward kernel for the VALU (paper, Sec. 3.2 batch-inner tiling and
// Sec. 3.3 mixed-precision storage, re-designed for gfx950).
//
// Work decomposition.  One 256-lane workgroup owns a voxel tile of 256 voxels
// (shape tx*ty*tz, one voxel per lane) and BT batch items.  Neighbouring
// voxels need nearby sample indices of every (transmit, element) channel
// (Sec. 3.1), so for each channel the workgroup stages one contiguous window
// of samples into LDS with coalesced loads from the batch-inner workspace
// ws[Q][M][K][B], and every lane then reads its two taps as one LDS access.
//
//   * Aperture culling: before the element loop the workgroup tests every
//     element's receive cone against the tile's bounding sphere and compacts
//     the elements that can have a nonzero weight into an LDS list; only
//     those are visited.  Inside a chunk, a wavefront skips an element when
//     all its 64 voxels have zero weight.
//   * Windows: the window of channel (q, m) starts at ktx_q + krx_m - dint,
//     where ktx_q + krx_m is the integer part of the tile reference index and
//     dint bounds |f - (ktx + krx)| over the tile (triangle inequality on the
//     tile diagonal).  Each LDS entry holds the pair (s(j), s(j+1)) so both taps
//     come from one read; taps outside [0, K) are zero-filled while staging.
//   * Loop order: element chunks (MC elements) outer, transmits inner; the
//     receive geometry and weight of a (voxel, element) pair are formed once
//     and reused across up to 16 transmits.
//   * Block ids are remapped so that each XCD (and its L2) receives a
//     contiguous range of tiles, whose windows overlap.
//
// Arithmetic: delays are tile-relative FP32 with FP64 reference terms
// (das_device.h); samples are converted to FP32 before interpolation and all
// accumulation is FP32.
#include "das_device.h"

namespace dasmi {
namespace {

constexpr int QG = 16;
constexpr int NT = 256;

template <class T> struct Pair;
template <> struct Pair<float> {
  using type = float2;
  __device__ static float2 make(float a, float b) { return make_float2(a, b); }
  __device__ static void split(float2 v, float& a, float& b) { a = v.x; b = v.y; }
};
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
template <> struct Pair<_Float16> {
  using type = half2_t;
  __device__ static void split(half2_t v, float& a, float& b) {
    a = (float)v.x;
    b = (float)v.y;
  }
};
template <> struct Pair<uint16_t> {
  using type = uint32_t;
  __device__ static void split(uint32_t v, float& a, float& b) {
    a = __uint_as_float(v << 16);
    b = __uint_as_float(v & 0xffff0000u);
  }
};

template <class T> __device__ inline typename Pair<T>::type make_pair(T a, T b);
template <> __device__ inline float2 make_pair<float>(float a, float b) { return make_float2(a, b); }
template <> __device__ inline half2_t make_pair<_Float16>(_Float16 a, _Float16 b) {
  half2_t v;
  v.x = a;
  v.y = b;
  return v;
}
template <> __device__ inline uint32_t make_pair<uint16_t>(uint16_t a, uint16_t b) {
  return (uint32_t)a | ((uint32_t)b << 16);
}

struct MInfo {  // per staged element, 32 bytes
  float ex, ey, ez, en, h;
  int krx, m, pad;
};
struct QInfo {  // per transmit of the current group, 32 bytes
  float vx, vy, vz, vn, g;
  int ktx, kind, pad;
};

template <int MC, class T>
__host__ __device__ constexpr size_t pairs_bytes(int P, int BT) {
  return ((size_t)QG * MC * P * BT * sizeof(typename Pair<T>::type) + 15) & ~(size_t)15;
}

template <class T, int BT, int MC, bool WTX>
__global__ __launch_bounds__(NT) void tiled_forward(Geom g, TileShape ts, Window win,
                                                    const T* __restrict__ ws, int B,
                                                    float* __restrict__ x, int ntx, int nty,
                                                    int ntiles, int per_xcd) {
  using PT = typename Pair<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  const int P = win.pairs;
  PT* pairs = reinterpret_cast<PT*>(smem);
  MInfo* minfo = reinterpret_cast<MInfo*>(smem + pairs_bytes<MC, T>(P, BT));
  QInfo* qinfo = reinterpret_cast<QInfo*>(minfo + MC);
  int* wcount = reinterpret_cast<int*>(qinfo + QG);           // [4]
  uint16_t* act = reinterpret_cast<uint16_t*>(wcount + 4);   // [M]

  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int tile = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (tile >= ntiles) return;
  const int tix = tile % ntx, tiy = (tile / ntx) % nty, tiz = tile / (ntx * nty);
  const int lx = t & (ts.tx - 1), ly = (t >> ts.lx) & (ts.ty - 1), lz = t >> ts.lxy;
  const int ix = tix * ts.tx + lx, iy = tiy * ts.ty + ly, iz = tiz * ts.tz + lz;
  const int b0 = blockIdx.y * BT;
  const int K = g.K, M = g.M;
  const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];

  const float hx = 0.5f * (ts.tx - 1), hy = 0.5f * (ts.ty - 1), hz = 0.5f * (ts.tz - 1);
  double px, py, pz;
  tile_ref_point(g, tix * ts.tx + (double)hx, tiy * ts.ty + (double)hy, tiz * ts.tz + (double)hz,
                 px, py, pz);
  const float dx = ((float)lx - hx) * (float)g.s[0];
  const float dy = ((float)ly - hy) * (float)g.s[1];
  const float dz = ((float)lz - hz) * (float)g.s[2];
  const float dp2 = dx * dx + dy * dy + dz * dz;
  const float fscf = (float)g.fsc;
  const bool inside = in_grid(g, ix, iy, iz);
  const int n = grid_index(g, ix, iy, iz);

  // ---- aperture culling: compact the elements that can reach this tile ----
  const int nact = cull_elements(g, px, py, pz, hx, hy, hz, wcount, act);

  float acc[BT];
#pragma unroll
  for (int b = 0; b < BT; ++b) acc[b] = 0.f;

  for (int q0 = 0; q0 < g.Q; q0 += QG) {
    const int qn = min(QG, g.Q - q0);
    __syncthreads();
    if (t < qn) {
      const TxRef r = make_tx_ref(g, q0 + t, px, py, pz);
      qinfo[t] = QInfo{r.vx, r.vy, r.vz, r.vn, r.g, r.ktx, r.kind, 0};
    }
    __syncthreads();
    float bq[QG];
    float wq[WTX ? QG : 1];
#pragma unroll
    for (int q = 0; q < QG; ++q) {
      bq[q] = 0.f;
      if (WTX) wq[WTX ? q : 0] = 0.f;
      if (q < qn) {
        const QInfo qi = qinfo[q];
        TxRef r;
        r.vx = qi.vx; r.vy = qi.vy; r.vz = qi.vz; r.vn = qi.vn; r.kind = qi.kind;
        bq[q] = fmaf(delta_tx(r, dx, dy, dz, dp2), fscf, qi.g);
        if (WTX) wq[WTX ? q : 0] = inside ? g.w_tx[(size_t)(q0 + q) * N + n] : 0.f;
      }
    }

    for (int c0 = 0; c0 < nact; c0 += MC) {
      const int mcn = min(MC, nact - c0);
      __syncthreads();  // the previous chunk is no longer read
      if (t < mcn) {
        const int m = act[c0 + t];
        const RxRef r = make_rx_ref(g, m, px, py, pz);
        minfo[t] = MInfo{r.ex, r.ey, r.ez, r.en, r.h, r.krx, m, 0};
      }
      __syncthreads();
      // ---- stage windows: wave w stages windows w, w+4, ... of the chunk ----
      for (int wi = wave; wi < QG * MC; wi += 4) {
        const int q = wi / MC, mc = wi % MC;
        if (q >= qn || mc >= mcn) continue;
        const int j0 = qinfo[q].ktx + minfo[mc].krx - win.dint;
        const T* src = ws + ((size_t)(q0 + q) * M + minfo[mc].m) * (size_t)K * B;
        PT* dst = pairs + (q * MC + mc) * P * BT;
        for (int p = lane; p < P; p += 64) {
          const int j = j0 + p;
#pragma unroll
          for (int b = 0; b < BT; ++b) {
            T s1 = T(0), s2 = T(0);
            if (b0 + b < B) {
              if (j >= 0 && j < K) s1 = src[(size_t)j * B + b0 + b];
              if (j + 1 >= 0 && j + 1 < K) s2 = src[(size_t)(j + 1) * B + b0 + b];
            }
            dst[p * BT + b] = make_pair<T>(s1, s2);
          }
        }
      }
      __syncthreads();
      // ---- interpolate and accumulate ----
      for (int mc = 0; mc < mcn; ++mc) {
        const MInfo mi = minfo[mc];
        const float ax = mi.ex + dx, ay = mi.ey + dy, az = mi.ez + dz;
        const float w = rx_weight(g, mi.m, ax, ay, az);
        if (__ballot(w != 0.f) == 0ull) continue;
        const float a = fmaf(delta_dist(mi.ex, mi.ey, mi.ez, mi.en, dx, dy, dz, dp2), fscf, mi.h);
        const PT* base = pairs + (mc * P + win.dint) * BT;
#pragma unroll
        for (int q = 0; q < QG; ++q) {
          if (q < qn) {
            const float f = a + bq[q];
            const float fl = floorf(f);
            const float al = f - fl;
            const int i = (int)fl;
            const float wt = WTX ? w * wq[WTX ? q : 0] : w;
            const PT* pp = base + (q * MC * P + i) * BT;
#pragma unroll
            for (int b = 0; b < BT; ++b) {
              float s1, s2;
              Pair<T>::split(pp[b], s1, s2);
              acc[b] = fmaf(wt, fmaf(al, s2, fmaf(-al, s1, s1)), acc[b]);
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

// Elements staged per chunk: the pair windows of a chunk take 16 transmits x
// 64 bytes x P, i.e. ~48 KiB at P = 47, so that three workgroups fit per CU.
template <class T, int BT>
constexpr int chunk_elems() {
  return (int)(64 / (BT * sizeof(typename Pair<T>::type))) < 1
             ? 1
             : (int)(64 / (BT * sizeof(typename Pair<T>::type)));
}

template <class T, int BT>
size_t lds_bytes_t(const Geom& g, const Window& w) {
  constexpr int MC = chunk_elems<T, BT>();
  size_t b = pairs_bytes<MC, T>(w.pairs, BT) + MC * sizeof(MInfo) + QG * sizeof(QInfo) + 16 +
             (size_t)g.M * 2;
  return (b + 15) & ~(size_t)15;
}

template <class T, int BT>
hipError_t tiled_t(const Geom& g, const TileShape& ts, const Window& w, const void* ws, int B,
                   float* x, hipStream_t st) {
  constexpr int MC = chunk_elems<T, BT>();
  const int ntx = (g.n[0] + ts.tx - 1) / ts.tx, nty = (g.n[1] + ts.ty - 1) / ts.ty,
            ntz = (g.n[2] + ts.tz - 1) / ts.tz;
  const int ntiles = ntx * nty * ntz;
  const int per_xcd = (ntiles + 7) / 8;
  const size_t lds = lds_bytes_t<T, BT>(g, w);
  dim3 grid(per_xcd * 8, (B + BT - 1) / BT);
  if (g.w_tx) {
    auto kern = tiled_forward<T, BT, MC, true>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, g, ts, w, static_cast<const T*>(ws), B, x,
                       ntx, nty, ntiles, per_xcd);
  } else {
    auto kern = tiled_forward<T, BT, MC, false>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, g, ts, w, static_cast<const T*>(ws), B, x,
                       ntx, nty, ntiles, per_xcd);
  }
  return hipGetLastError();
}

template <class T>
hipError_t tiled_dispatch(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                          int B, float* x, hipStream_t st) {
  const int bt = tiled_batch_per_thread(sizeof(T) == 4 ? DAS_STORE_F32 : DAS_STORE_F16, B);
  if (bt == 4) return tiled_t<T, 4>(g, ts, w, ws, B, x, st);
  if (bt == 2) return tiled_t<T, 2>(g, ts, w, ws, B, x, st);
  return tiled_t<T, 1>(g, ts, w, ws, B, x, st);
}

}  // namespace

int tiled_batch_per_thread(int storage, int B) {
  (void)storage;
  if (B >= 4) return 4;
  if (B >= 2) return 2;
  return 1;
}

size_t tiled_lds_bytes(const Geom& g, int storage, int bt, const Window& w) {
  if (storage == DAS_STORE_F32) {
    if (bt == 4) return lds_bytes_t<float, 4>(g, w);
    if (bt == 2) return lds_bytes_t<float, 2>(g, w);
    return lds_bytes_t<float, 1>(g, w);
  }
  if (bt == 4) return lds_bytes_t<_Float16, 4>(g, w);
  if (bt == 2) return lds_bytes_t<_Float16, 2>(g, w);
  return lds_bytes_t<_Float16, 1>(g, w);
}

hipError_t launch_tiled_forward(const Geom& g, int storage, const TileShape& ts, const Window& w,
                                const void* ws, int B, float* x, hipStream_t st) {
  switch (storage) {
    case DAS_STORE_F32: return tiled_dispatch<float>(g, ts, w, ws, B, x, st);
    case DAS_STORE_F16: return tiled_dispatch<_Float16>(g, ts, w, ws, B, x, st);
    default: return tiled_dispatch<uint16_t>(g, ts, w, ws, B, x, st);
  }
}

}  // namespace dasmi
