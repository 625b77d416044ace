// Windowed forward kernel for the VALU (paper, Sec. 3.2 batch-inner tiling and
// Sec. 3.3 mixed-precision storage, re-designed for gfx950).
//
// Work decomposition.  One 256-lane workgroup owns a voxel tile of 256 voxels
// (shape tx*ty*tz, one voxel per lane; each 64-lane wavefront owns a box of 64
// of them) and BT batch items.  Neighbouring voxels need nearby sample indices
// of every (transmit, element) channel (Sec. 3.1), so for each channel the
// workgroup stages one contiguous window of samples into LDS with coalesced
// loads from the batch-inner workspace ws[Q][M][K][B], converted to FP32, and
// every lane then reads its two taps with one ds_read2_b32.
//
//   * Tile set-up: every element is tested against the receive-aperture cone
//     (a conservative sphere-cone test for the tile and for each wavefront's
//     box).  The elements that can reach the tile are compacted into an LDS
//     list with their FP64 reference terms (tile-relative delays, see
//     das_device.h) and a 4-bit mask of the wavefronts they can reach; a
//     wavefront skips an element of the list with one bit test.
//   * Windows: the window of channel (q, m) starts at ktx_q + krx_m - dint,
//     where ktx_q + krx_m is the integer part of the tile reference index and
//     dint bounds |f - (ktx + krx)| over the tile (triangle inequality on the
//     tile half-diagonal).  Taps outside [0, K) are zero-filled while staging.
//   * Pipelining: element chunks (MC elements x QN transmits) are staged
//     through registers: the global loads of chunk c+1 are issued before the
//     interpolation of chunk c and written to LDS after it, so memory latency
//     hides behind arithmetic.
//   * Loop order: element chunks outer, transmits inner; the receive geometry
//     and weight of a (voxel, element) pair are formed once and reused across
//     the QN transmits of a group, whose QN LDS reads are all issued before
//     the first is consumed.
//   * Tiles are dispatched deepest layer first: the cost of a tile grows with
//     the number of elements whose aperture reaches it (with depth, for an
//     f-number aperture), so the longest tiles start first and the short
//     ones fill the tail; consecutive block ids land on different XCDs, so
//     every XCD receives the same mix of depths.
//
// Arithmetic: delays are tile-relative FP32 with FP64 reference terms;
// samples are converted to FP32 before interpolation; accumulation is FP32.
// Transmits are processed in groups of QN (compile-time, so the transmit loop
// unrolls); a group that is not full is padded with zero-filled windows.
#pragma once
#include "das_device.h"
#include "fp8.h"

namespace dasmi {
namespace tiled {

constexpr int NT = 256;
constexpr int EMAX = 512;  // active elements held per pass
constexpr int WS = 64;     // samples per window slot; windows hold W <= WS
// LDS windows of a chunk are stored [mc][sample][q] with the transmit index
// innermost and the row padded to QN + 1 entries: the two taps of transmit q
// are then one ds_read2 with offsets q and q + QN + 1 from a per-lane address,
// and staging writes of consecutive samples do not collide in one bank.
template <int QN> struct Row { static constexpr int QP = QN + 1; };
// Floats between consecutive samples of a window: QP entries of BT items,
// plus 4 for eight items (136 floats would put samples 8 rows apart on the
// same LDS banks).
__host__ __device__ constexpr int row_stride(int QN, int BT) { return (QN + 1) * BT + (BT == 8 ? 4 : 0); }

template <class T> __device__ inline float to_f32(T v);
template <> __device__ inline float to_f32<float>(float v) { return v; }
template <> __device__ inline float to_f32<_Float16>(_Float16 v) { return (float)v; }
template <> __device__ inline float to_f32<uint16_t>(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);
}
template <> __device__ inline float to_f32<uint8_t>(uint8_t v) {  // FP8 E4M3 code
  return e4m3_to_f32(v);
}

// Elements per chunk: QN * MC * BT = 64 windows of at most 64 samples
// (16 KiB of LDS at most; 16 staging registers per lane).
template <int BT, int QN>
constexpr int chunk_elems() {
  return 64 / (QN * BT) < 1 ? 1 : 64 / (QN * BT);
}

struct QInfo {  // per transmit of the current group, 32 bytes
  float vx, vy, vz, vn, g;
  int ktx, kind;
  int rq;  // complex baseband: the transmit's phase term (float bits, revolutions)
};

// LDS layout (bytes), shared by the kernel and the host-side size query.
struct Layout {
  int win, ex, ey, ez, eh, en, ek, em, q, wc, total;
};
__host__ __device__ inline Layout layout(int QN, int MC, int BT, int W) {
  Layout L;
  L.win = 0;
  (void)W;
  int o = ((MC * WS * row_stride(QN, BT) * 4) + 15) & ~15;
  L.ex = o; o += EMAX * 4;
  L.ey = o; o += EMAX * 4;
  L.ez = o; o += EMAX * 4;
  L.eh = o; o += EMAX * 4;
  L.en = o; o += EMAX * 4;
  L.ek = o; o += EMAX * 4;
  L.em = o; o += EMAX * 4;
  L.q = o; o += 16 * (int)sizeof(QInfo);
  L.wc = o; o += 16;
  L.total = o;
  return L;
}

// Conservative test: can any point of the sphere (centre c, radius R) lie in
// the open receive cone of element m (apex r_m, axis n_m, half-angle theta
// with tan theta = 1/(2F))?  With D = |c - r_m|, cos(phi) = (c - r_m).n / D
// and beta = asin(R/D), the sphere meets the cone iff phi < theta + beta, i.e.
// cos(phi) > cos(theta) cos(beta) - sin(theta) sin(beta) (when theta + beta
// < pi, which holds here since theta < pi/2 and beta <= pi/2).
__device__ inline bool sphere_meets_cone(float ex, float ey, float ez, float nx, float ny,
                                         float nz, float R, float cth, float sth) {
  const float D2 = ex * ex + ey * ey + ez * ez;
  const float R2 = R * R * 1.0001f + 1e-18f;
  if (D2 <= R2) return true;
  const float invD = __builtin_amdgcn_rsqf(D2);
  const float cphi = (ex * nx + ey * ny + ez * nz) * invD;
  const float sb = R * invD;
  const float cb = __builtin_amdgcn_sqrtf(fmaxf(0.f, 1.f - sb * sb));
  return cphi > cth * cb - sth * sb - 1e-4f;
}

// Per-thread staging registers for one chunk: lane p of wave w holds sample
// p of windows w, w+4, ... (BT batch items each).
template <int BT, int QN, int MC>
struct Stage {
  static constexpr int WPW = (QN * MC + 3) / 4;
  float v[WPW][BT];
};

template <class T, int BT, int QN, int MC>
__device__ inline void stage_load(Stage<BT, QN, MC>& st, const T* __restrict__ ws, const int* ktx,
                                  const int* ek, const int* em, const int* txl, int c0, int q0,
                                  int qn, int mcn, int M, int K, int B, int b0, int W, int dint,
                                  int wave, int lane) {
  constexpr int WPW = Stage<BT, QN, MC>::WPW;
#pragma unroll
  for (int k = 0; k < WPW; ++k) {
    const int wi = wave + 4 * k;
    const int q = wi / MC, mc = wi % MC;
    // 16- and 8-bit codes stay packed (the first BT sizeof(T) / 4 slots)
    // until the LDS store converts them
    T u[BT];
#pragma unroll
    for (int b = 0; b < BT; ++b) u[b] = T(0);
    if (wi < QN * MC && q < qn && mc < mcn) {
      // window (q, mc) is wavefront-uniform: scalar base, 32-bit lane offset
      const int e = c0 + mc;
      const int krx = __builtin_amdgcn_readfirstlane(ek[e]);
      const int m = __builtin_amdgcn_readfirstlane(em[e]) & 0xffff;
      const int j0 = __builtin_amdgcn_readfirstlane(ktx[q]) + krx - dint;
      const int qt = txl ? __builtin_amdgcn_readfirstlane(txl[q0 + q]) : q0 + q;  // transmit
      const T* chan = ws + ((size_t)qt * M + m) * (size_t)K * B + b0;
      const int j = j0 + lane;
      if (lane < W && j >= 0 && j < K) {
        const T* src = chan + (size_t)j * B;
        // the BT items of a sample are contiguous (batch-inner): one vector
        // load when they are all present and aligned
        if (BT > 1 && b0 + BT <= B && (reinterpret_cast<uintptr_t>(src) & (BT * sizeof(T) - 1)) == 0) {
          typedef T vecT __attribute__((ext_vector_type(BT)));
          const vecT uv = *reinterpret_cast<const vecT*>(src);
#pragma unroll
          for (int b = 0; b < BT; ++b) u[b] = uv[b];
        } else {
#pragma unroll
          for (int b = 0; b < BT; ++b)
            if (b0 + b < B) u[b] = src[b];
        }
      }
    }
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int b = 0; b < BT; ++b) st.v[k][b] = to_f32<T>(u[b]);
    } else {
      constexpr int NW = (BT * (int)sizeof(T) + 3) / 4;
      uint32_t w[NW];
#pragma unroll
      for (int i = 0; i < NW; ++i) w[i] = 0u;
      __builtin_memcpy(w, u, sizeof(u));
#pragma unroll
      for (int i = 0; i < NW; ++i) st.v[k][i] = __uint_as_float(w[i]);
    }
  }
}

// Item b of staged window slot k as FP32 (see stage_load).
template <class T, int BT, int QN, int MC>
__device__ inline float staged_item(const Stage<BT, QN, MC>& st, int k, int b) {
  if constexpr (sizeof(T) == 4) {
    return st.v[k][b];
  } else {
    constexpr int NW = (BT * (int)sizeof(T) + 3) / 4;
    uint32_t w[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = __float_as_uint(st.v[k][i]);
    T u[BT];
    __builtin_memcpy(u, w, sizeof(u));
    return to_f32<T>(u[b]);
  }
}

template <class T, int BT, int QN, int MC>
__device__ inline void stage_store(const Stage<BT, QN, MC>& st, float* win, int mcn, int W,
                                   int wave, int lane) {
  constexpr int WPW = Stage<BT, QN, MC>::WPW;
#pragma unroll
  for (int k = 0; k < WPW; ++k) {
    const int wi = wave + 4 * k;
    const int q = wi / MC, mc = wi % MC;
    if (wi < QN * MC && mc < mcn && lane < W) {
      float* dst = win + (mc * WS + lane) * row_stride(QN, BT) + q * BT;
#pragma unroll
      for (int b = 0; b < BT; ++b) dst[b] = staged_item<T, BT, QN, MC>(st, k, b);
    }
  }
}

// Single-item workspaces (B = 1, the headline case) stage windows four
// samples per lane: samples of a window are contiguous in ws[Q][M][K], so 16
// lanes cover a 64-sample window with one load of four samples each (16, 8 or
// 4 bytes), a wavefront four windows per instruction (a quarter of the
// address work of one sample per lane).  The LDS layout stays
// [mc][sample][q] (the taps of all transmits of a lane one immediate offset
// apart); the four samples go out as four stores.  The four window groups of an instruction take consecutive
// transmits of one element (q = wi mod QN), so their stores land one bank
// apart; taking consecutive elements instead puts all four groups on the
// same banks (an element is WS * QP words, a multiple of the bank count).
// The layout must be [Q][M][K] (a plan of one item): a persistent launch can
// run its one-item-per-thread body over plans of several items, so the
// choice is made at run time on the plan's batch (the staging registers are
// shared: Stage<1, QN, MC> holds 16 floats, four rounds of four samples).
template <class T, int BT>
constexpr bool kVecStage = BT == 1;

// Lane -> (window group g, first sample s): lanes 8g .. 8g+7 take samples
// 0 .. 31 of window g and lanes 32+8g .. 32+8g+7 samples 32 .. 63, so each
// half-wavefront (the LDS serves 32 lanes a cycle) stores 4 windows x 8
// quads, banks 4j + g: all 32 distinct.
__device__ inline int vec_group(int lane) { return (lane >> 3) & 3; }
__device__ inline int vec_sample(int lane) { return 4 * ((lane & 7) | ((lane >> 5) << 3)); }

template <class T, int QN, int MC>
__device__ inline void stage_load4(Stage<1, QN, MC>& st, const T* __restrict__ ws, const int* ktx,
                                   const int* ek, const int* em, const int* txl, int c0, int q0,
                                   int qn, int mcn, int M, int K, int W, int dint, int wave,
                                   int lane) {
  const int s = vec_sample(lane);  // first sample of this lane within its window
  static_assert(Stage<1, QN, MC>::WPW == 16, "64 windows per chunk");
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int wi = 16 * k + 4 * wave + vec_group(lane);
    const int q = wi % QN, mc = wi / QN;
    float4 v = {0.f, 0.f, 0.f, 0.f};
    if (q < qn && mc < mcn && s < W) {
      const int e = c0 + mc;
      const int m = em[e] & 0xffff;
      const int j = ktx[q] + ek[e] - dint + s;
      const int qt = txl ? txl[q0 + q] : q0 + q;
      // qt M + m < 2^28 (Q <= 4096, M <= 65535): one 32 x 32 -> 64-bit product
      const T* chan = ws + (size_t)(unsigned)(qt * M + m) * (unsigned)K;
      if constexpr (sizeof(T) < 4) {
        // 16- and 8-bit codes stay packed in the staging registers (two or
        // one of the four slots) and are converted at the LDS store: half
        // or a quarter of the registers held across the interpolation
        T u[4];
        if (j >= 0 && j + 3 < K) {
          __builtin_memcpy(u, chan + j, sizeof(u));
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) u[i] = (j + i >= 0 && j + i < K) ? chan[j + i] : T(0);
        }
        uint32_t w[2] = {0u, 0u};
        __builtin_memcpy(w, u, sizeof(u));
        v.x = __uint_as_float(w[0]);
        v.y = __uint_as_float(w[1]);
      } else if (j >= 0 && j + 3 < K) {
        T u[4];
        __builtin_memcpy(u, chan + j, sizeof(u));
        v = float4{to_f32<T>(u[0]), to_f32<T>(u[1]), to_f32<T>(u[2]), to_f32<T>(u[3])};
      } else {
        v.x = (j >= 0 && j < K) ? to_f32<T>(chan[j]) : 0.f;
        v.y = (j + 1 >= 0 && j + 1 < K) ? to_f32<T>(chan[j + 1]) : 0.f;
        v.z = (j + 2 >= 0 && j + 2 < K) ? to_f32<T>(chan[j + 2]) : 0.f;
        v.w = (j + 3 >= 0 && j + 3 < K) ? to_f32<T>(chan[j + 3]) : 0.f;
      }
    }
    st.v[4 * k + 0][0] = v.x;
    st.v[4 * k + 1][0] = v.y;
    if constexpr (sizeof(T) == 4) {
      st.v[4 * k + 2][0] = v.z;
      st.v[4 * k + 3][0] = v.w;
    }
  }
}

// The four staged samples of slot group k as FP32 (see stage_load4).
template <class T, int QN, int MC>
__device__ inline float4 staged4(const Stage<1, QN, MC>& st, int k) {
  if constexpr (sizeof(T) == 4) {
    return float4{st.v[4 * k][0], st.v[4 * k + 1][0], st.v[4 * k + 2][0], st.v[4 * k + 3][0]};
  } else {
    const uint32_t w[2] = {__float_as_uint(st.v[4 * k][0]), __float_as_uint(st.v[4 * k + 1][0])};
    T u[4];
    __builtin_memcpy(u, w, sizeof(u));
    return float4{to_f32<T>(u[0]), to_f32<T>(u[1]), to_f32<T>(u[2]), to_f32<T>(u[3])};
  }
}

template <class T, int QN, int MC>
__device__ inline void stage_store4(const Stage<1, QN, MC>& st, float* win, int mcn, int W,
                                    int wave, int lane) {
  const int s = vec_sample(lane);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int wi = 16 * k + 4 * wave + vec_group(lane);
    const int q = wi % QN, mc = wi / QN;
    constexpr int QP = Row<QN>::QP;
    if (mc < mcn && s < W) {
      const float4 v = staged4<T, QN, MC>(st, k);
      float* dst = win + (mc * WS + s) * QP + q;
      dst[0] = v.x;
      if (s + 1 < W) dst[QP] = v.y;
      if (s + 2 < W) dst[2 * QP] = v.z;
      if (s + 3 < W) dst[3 * QP] = v.w;
    }
  }
}

// One tile (tile index `tile`, batch items b0 .. b0+BT-1) of the windowed
// forward; all 256 threads of the workgroup call it together.
// RUNTIME_VEC: the one-item staging path is chosen per plan at run time (the
// persistent kernel, whose one-item-per-thread body may serve plans of
// several items); otherwise BT == 1 implies a one-item plan.
// CUBIC: four-point Lagrange interpolation through samples k-1 .. k+2 instead
// of the linear interpolation of Eq. (2) (the paper allows other schemes); the
// window of a tile already holds those taps (tap i = floor(f) + dint lies in
// [1, 2 dint + 1] and the window has 2 dint + 4 samples).
template <class T, int BT, int QN, bool WTX, bool IQ = false, bool RUNTIME_VEC = false,
          bool CUBIC = false>
__device__ inline void tile_body(const Geom& g, const TileShape& ts, const Window& win,
                                 const T* __restrict__ ws, int B, float* __restrict__ x, int ntx,
                                 int nty, int ntiles, int tile, int b0, unsigned char* smem,
                                 int* ktx_s, int* txl_s) {
  constexpr int MC = chunk_elems<BT, QN>();
  const int W = win.pairs + 1;  // samples per window
  const Layout L = layout(QN, MC, BT, W);
  float* wsm = reinterpret_cast<float*>(smem + L.win);
  float* eX = reinterpret_cast<float*>(smem + L.ex);
  float* eY = reinterpret_cast<float*>(smem + L.ey);
  float* eZ = reinterpret_cast<float*>(smem + L.ez);
  float* eH = reinterpret_cast<float*>(smem + L.eh);
  float* eN = reinterpret_cast<float*>(smem + L.en);
  int* eK = reinterpret_cast<int*>(smem + L.ek);
  int* eM = reinterpret_cast<int*>(smem + L.em);
  QInfo* qinfo = reinterpret_cast<QInfo*>(smem + L.q);
  int* wcount = reinterpret_cast<int*>(smem + L.wc);

  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int ntz = ntiles / (ntx * nty);
  const int tix = tile % ntx, tiy = (tile / ntx) % nty, tiz = ntz - 1 - tile / (ntx * nty);
  // wavefront `wave` covers box (bx, by, bz) of the tile, x fastest inside
  const int bxi = wave & (ts.bx - 1), byi = (wave >> ts.blx) & (ts.by - 1), bzi = wave >> ts.blxy;
  const int lx = bxi * ts.wx + (lane & (ts.wx - 1));
  const int ly = byi * ts.wy + ((lane >> ts.wlx) & (ts.wy - 1));
  const int lz = bzi * ts.wz + (lane >> ts.wlxy);
  const int ix = tix * ts.tx + lx, iy = tiy * ts.ty + ly, iz = tiz * ts.tz + lz;
  const int K = g.K, M = g.M;
  const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];

  const float hx = 0.5f * (ts.tx - 1), hy = 0.5f * (ts.ty - 1), hz = 0.5f * (ts.tz - 1);
  double px, py, pz;
  tile_ref_point(g, tix * ts.tx + (double)hx, tiy * ts.ty + (double)hy, tiz * ts.tz + (double)hz,
                 px, py, pz);
  const float sx = (float)g.s[0], sy = (float)g.s[1], sz = (float)g.s[2];
  const float dx = ((float)lx - hx) * sx, dy = ((float)ly - hy) * sy, dz = ((float)lz - hz) * sz;
  const float dp2 = dx * dx + dy * dy + dz * dz;
  const float fscf = (float)g.fsc;
  const bool inside = in_grid(g, ix, iy, iz);
  const int n = grid_index(g, ix, iy, iz);
  const uint32_t mybit = 1u << (16 + wave);

  // Bounding spheres (relative to the tile reference) of the tile and of the
  // four wavefront boxes.
  const float Rt = sqrtf(hx * hx * sx * sx + hy * hy * sy * sy + hz * hz * sz * sz);
  float wcx[4], wcy[4], wcz[4], wr[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const float ax0 = (float)((w & (ts.bx - 1)) * ts.wx);
    const float ay0 = (float)(((w >> ts.blx) & (ts.by - 1)) * ts.wy);
    const float az0 = (float)((w >> ts.blxy) * ts.wz);
    const float ax1 = ax0 + (float)(ts.wx - 1), ay1 = ay0 + (float)(ts.wy - 1),
                az1 = az0 + (float)(ts.wz - 1);
    wcx[w] = (0.5f * (ax0 + ax1) - hx) * sx;
    wcy[w] = (0.5f * (ay0 + ay1) - hy) * sy;
    wcz[w] = (0.5f * (az0 + az1) - hz) * sz;
    wr[w] = 0.5f * sqrtf((ax1 - ax0) * (ax1 - ax0) * sx * sx + (ay1 - ay0) * (ay1 - ay0) * sy * sy +
                         (az1 - az0) * (az1 - az0) * sz * sz);
  }
  const bool hann = g.apod == DAS_APOD_HANN_FNUM;
  const float twoF = sqrtf(g.fourF2);
  const float cth = hann ? twoF * rsqrtf(1.f + g.fourF2) : -1.f;
  const float sth = hann ? rsqrtf(1.f + g.fourF2) : 0.f;

  float acc[BT];
#pragma unroll
  for (int b = 0; b < BT; ++b) acc[b] = 0.f;

  // Sparse transmit list (the paper's sparse observation lists, Sec. 5): with
  // transmit weights and Q <= 64 the tile loops only over the transmits whose
  // weight is nonzero somewhere in it (txl_s[0 .. nq-1]); every term skipped
  // is an exact zero, so the result does not change.
  int nq = g.Q;
  const int* txl = nullptr;
  if (WTX && g.Q <= 64) {
    uint64_t mine = 0;
    if (inside)
      for (int q = 0; q < g.Q; ++q)
        if (g.w_tx[(size_t)q * N + n] != 0.f) mine |= 1ull << q;
    uint32_t lo = (uint32_t)mine, hi = (uint32_t)(mine >> 32);
    for (int o = 32; o > 0; o >>= 1) {
      lo |= (uint32_t)__shfl_xor((int)lo, o);
      hi |= (uint32_t)__shfl_xor((int)hi, o);
    }
    __syncthreads();  // txl_s is free (a previous tile of a persistent launch is done)
    if (lane == 0) {
      txl_s[64 + 2 * wave] = (int)lo;
      txl_s[65 + 2 * wave] = (int)hi;
    }
    __syncthreads();
    uint64_t all = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w)
      all |= (uint64_t)(uint32_t)txl_s[64 + 2 * w] | ((uint64_t)(uint32_t)txl_s[65 + 2 * w] << 32);
    if (t < g.Q && ((all >> t) & 1ull)) txl_s[__popcll(all & ((1ull << t) - 1ull))] = t;
    nq = __popcll(all);
    txl = txl_s;
    // the list is published by the barrier at the start of the transmit-group loop
  }

  int mscan = 0;
  while (mscan < M) {
    // ---- compact the next batch of elements that can reach this tile ----
    int nact = 0;
    __syncthreads();
    while (mscan < M && nact + NT <= EMAX) {
      const int m = mscan + t;
      uint32_t mask = 0;
      double ex = 0.0, ey = 0.0, ez = 0.0;
      if (m < M) {
        ex = px - g.elem[3 * m + 0];
        ey = py - g.elem[3 * m + 1];
        ez = pz - g.elem[3 * m + 2];
        if (!hann) {
          mask = 0xfu;
        } else {
          float nx = 0.f, ny = 0.f, nz = 1.f;
          if (g.enorm) {
            nx = g.enorm[3 * m + 0];
            ny = g.enorm[3 * m + 1];
            nz = g.enorm[3 * m + 2];
          }
          const float fx = (float)ex, fy = (float)ey, fz = (float)ez;
          if (sphere_meets_cone(fx, fy, fz, nx, ny, nz, Rt, cth, sth)) {
#pragma unroll
            for (int w = 0; w < 4; ++w)
              if (sphere_meets_cone(fx + wcx[w], fy + wcy[w], fz + wcz[w], nx, ny, nz, wr[w], cth, sth))
                mask |= 1u << w;
          }
        }
      }
      const bool on = mask != 0;
      const uint64_t bal = __ballot(on);
      const int before = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) wcount[wave] = __popcll(bal);
      __syncthreads();
      int off = nact;
      for (int w = 0; w < wave; ++w) off += wcount[w];
      if (on) {
        const int e = off + before;
        const double R = sqrt(ex * ex + ey * ey + ez * ez);
        const double fr = R * g.fsc;
        const double fl = floor(fr);
        const float fx = (float)ex, fy = (float)ey, fz = (float)ez;
        eX[e] = fx;
        eY[e] = fy;
        eZ[e] = fz;
        eH[e] = (float)(fr - fl);
        eN[e] = __builtin_amdgcn_sqrtf(fx * fx + fy * fy + fz * fz);  // |r_m - p_tile|, FP32
        eK[e] = (int)fl;
        eM[e] = (int)(m | (mask << 16));
      }
      nact += wcount[0] + wcount[1] + wcount[2] + wcount[3];
      mscan += NT;
      __syncthreads();
    }

    for (int q0 = 0; q0 < nq; q0 += QN) {
      const int qn = min(QN, nq - q0);
      __syncthreads();
      if (t < qn) {
        const TxRef r = make_tx_ref(g, txl ? txl[q0 + t] : q0 + t, px, py, pz);
        // complex baseband: the transmit's phase term frac(fc/fs ktx + fc t0)
        // in revolutions (FP64 before rounding: ktx reaches thousands)
        int rq_bits = 0;
        if constexpr (IQ) {
          const double rv = g.fcfs * (double)r.ktx + g.fct0;
          rq_bits = __float_as_int((float)(rv - floor(rv)));
        }
        qinfo[t] = QInfo{r.vx, r.vy, r.vz, r.vn, r.g, r.ktx, r.kind, rq_bits};
        ktx_s[t] = r.ktx;
      }
      __syncthreads();
      float bq[QN];
      float wq[WTX ? QN : 1];
      // complex baseband: the phase of a term splits into a transmit part
      // (frac(fc/fs ktx + fc t0) + fc/fs bq) and an element part (frac(fc/fs
      // krx) + fc/fs a); each is turned into a unit phasor once (per transmit
      // of the group, per element) and a term's phasor is their product
      float pcq[IQ ? QN : 1], psq[IQ ? QN : 1];
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        bq[q] = 0.f;
        if (WTX) wq[WTX ? q : 0] = 0.f;
        if (IQ) pcq[IQ ? q : 0] = psq[IQ ? q : 0] = 0.f;
        if (q < qn) {
          const QInfo qi = qinfo[q];
          TxRef r;
          r.vx = qi.vx; r.vy = qi.vy; r.vz = qi.vz; r.vn = qi.vn; r.kind = qi.kind;
          bq[q] = fmaf(delta_tx(r, dx, dy, dz, dp2), fscf, qi.g);
          if constexpr (IQ) {
            // revolutions, reduced to [0, 1) before the hardware sine and
            // cosine (which take revolutions)
            const float rev = frac_f32(fmaf((float)g.fcfs, bq[q], __int_as_float(qi.rq)));
            pcq[q] = __builtin_amdgcn_cosf(rev);
            psq[q] = __builtin_amdgcn_sinf(rev);
          }
          if (WTX)
            wq[WTX ? q : 0] = !inside ? 0.f : g.w_tx[(size_t)(txl ? txl[q0 + q] : q0 + q) * N + n];
        }
      }

      const bool vec = kVecStage<T, BT> && (!RUNTIME_VEC || B == 1);  // uniform
      Stage<BT, QN, MC> st;
      if (nact > 0) {
        if constexpr (kVecStage<T, BT>) {
          if (vec)
            stage_load4<T, QN, MC>(st, ws, ktx_s, eK, eM, txl, 0, q0, qn, min(MC, nact), M, K, W,
                                   win.dint, wave, lane);
          else
            stage_load<T, BT, QN, MC>(st, ws, ktx_s, eK, eM, txl, 0, q0, qn, min(MC, nact), M, K,
                                      B, b0, W, win.dint, wave, lane);
        } else {
          stage_load<T, BT, QN, MC>(st, ws, ktx_s, eK, eM, txl, 0, q0, qn, min(MC, nact), M, K, B,
                                    b0, W, win.dint, wave, lane);
        }
      }
      for (int c0 = 0; c0 < nact; c0 += MC) {
        const int mcn = min(MC, nact - c0);
        __syncthreads();  // the previous chunk is no longer read
        if constexpr (kVecStage<T, BT>) {
          if (vec)
            stage_store4<T, QN, MC>(st, wsm, mcn, W, wave, lane);
          else
            stage_store<T, BT, QN, MC>(st, wsm, mcn, W, wave, lane);
        } else {
          stage_store<T, BT, QN, MC>(st, wsm, mcn, W, wave, lane);
        }
        __syncthreads();
        if (c0 + MC < nact) {
          bool done = false;
          if constexpr (kVecStage<T, BT>) {
            if (vec) {
              stage_load4<T, QN, MC>(st, ws, ktx_s, eK, eM, txl, c0 + MC, q0, qn,
                                     min(MC, nact - c0 - MC), M, K, W, win.dint, wave, lane);
              done = true;
            }
          }
          if (!done)
            stage_load<T, BT, QN, MC>(st, ws, ktx_s, eK, eM, txl, c0 + MC, q0, qn,
                                      min(MC, nact - c0 - MC), M, K, B, b0, W, win.dint, wave, lane);
        }
        // ---- interpolate and accumulate ----
        for (int mc = 0; mc < mcn; ++mc) {
          const int e = c0 + mc;
          const int mm = __builtin_amdgcn_readfirstlane(eM[e]);
          if (!(mm & mybit)) continue;  // scalar branch
          const float ex = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(eX[e])));
          const float ey = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(eY[e])));
          const float ez = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(eZ[e])));
          const float eh = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(eH[e])));
          const float ax = ex + dx, ay = ey + dy, az = ez + dz;
          const float w = rx_weight(g, mm & 0xffff, ax, ay, az);
          const float en = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(eN[e])));
          const float a = fmaf(delta_dist(ex, ey, ez, en, dx, dy, dz, dp2), fscf, eh);
          // complex baseband: the element's phasor, from frac(fc/fs krx)
          // (FP64 before rounding: krx reaches thousands) + fc/fs a
          float pcm = 1.f, psm = 0.f;
          if constexpr (IQ) {
            const double rv = g.fcfs * (double)__builtin_amdgcn_readfirstlane(eK[e]);
            const float rev = frac_f32(fmaf((float)g.fcfs, a, (float)(rv - floor(rv))));
            pcm = __builtin_amdgcn_cosf(rev);
            psm = __builtin_amdgcn_sinf(rev);
          }
          // tap index i = floor(f) + dint is in [1, 2 dint + 1] (window bound)
          constexpr int RS = row_stride(QN, BT);
          const float* base = wsm + (mc * WS + win.dint) * RS;
          // transmits per unit of the tap loop: eight one-item taps, or four
          // with transmit weights, whose sparse lists are short (the loop
          // stops after the unit holding the list's last transmit)
          constexpr int QR0 = QN * BT <= 8 ? QN : (8 / BT < 1 ? 1 : 8 / BT);
          constexpr int QR = WTX && QR0 > 4 ? 4 : QR0;
          // one group of QG transmits starting at qa: all tap reads first,
          // then the interpolation and accumulation
          auto taps = [&](auto qg_tag, int qa) {
            constexpr int QG = decltype(qg_tag)::value;
            constexpr int QC = CUBIC ? QG : 1;
            float s1[QG][BT], s2[QG][BT], al[QG];
            float s0[QC][BT], s3[QC][BT];
#pragma unroll
            for (int r = 0; r < QG; ++r) {
              const float f = a + bq[qa + r];
              al[r] = frac_f32(f);
              const float* pp = base + (__mul24(floor_i32(f), RS) + (qa + r) * BT);
#pragma unroll
              for (int b = 0; b < BT; ++b) {
                s1[r][b] = pp[b];
                s2[r][b] = pp[RS + b];
                if constexpr (CUBIC) {
                  s0[r][b] = pp[b - RS];
                  s3[r][b] = pp[2 * RS + b];
                }
              }
            }
            __builtin_amdgcn_sched_barrier(0);  // all reads of the group issue first
#pragma unroll
            for (int r = 0; r < QG; ++r) {
              const float wt = WTX ? w * wq[WTX ? qa + r : 0] : w;
              if constexpr (CUBIC) {
                // Lagrange weights of samples k-1, k, k+1, k+2 at k + alpha
                const float u = al[r], up = u + 1.f, um = u - 1.f, u2 = u - 2.f;
                const float uum = u * um, upu2 = up * u2;
                const float cm = uum * u2 * (-1.f / 6.f), c0 = upu2 * um * 0.5f;
                const float c1 = upu2 * u * -0.5f, c2 = uum * up * (1.f / 6.f);
#pragma unroll
                for (int b = 0; b < BT; ++b)
                  acc[b] = fmaf(wt, fmaf(cm, s0[r][b], fmaf(c0, s1[r][b], fmaf(c1, s2[r][b], c2 * s3[r][b]))),
                                acc[b]);
              } else if constexpr (IQ) {
                // remodulate by exp(i 2 pi fc tau), the product of the
                // transmit's and the element's phasors
                const float cs = fmaf(pcq[qa + r], pcm, -psq[qa + r] * psm);
                const float sn = fmaf(psq[qa + r], pcm, pcq[qa + r] * psm);
#pragma unroll
                for (int b = 0; b < BT; b += 2) {
                  const float vi = fmaf(al[r], s2[r][b], fmaf(-al[r], s1[r][b], s1[r][b]));
                  const float vq = fmaf(al[r], s2[r][b + 1], fmaf(-al[r], s1[r][b + 1], s1[r][b + 1]));
                  acc[b] = fmaf(wt, fmaf(cs, vi, -sn * vq), acc[b]);
                  acc[b + 1] = fmaf(wt, fmaf(sn, vi, cs * vq), acc[b + 1]);
                }
              } else {
#pragma unroll
                for (int b = 0; b < BT; ++b)
                  acc[b] = fmaf(wt, fmaf(al[r], s2[r][b], fmaf(-al[r], s1[r][b], s1[r][b])), acc[b]);
              }
            }
          };
          // with transmit weights the group may be short (sparse list): stop
          // at its last transmit (block-uniform); a list of at most four
          // transmits (the common case of selective weights) takes one
          // four-transmit group instead of a full one
#pragma unroll
          for (int qa = 0; qa < QN; qa += QR) {
            if (WTX && qa >= qn) break;  // block-uniform
            taps(std::integral_constant<int, QR>(), qa);
          }
        }
      }
    }
  }
  if (inside) {
#pragma unroll
    for (int b = 0; b < BT; ++b)
      if (b0 + b < B) {
        if constexpr (__is_same(T, uint8_t))  // FP8: the item was stored as y 2^e
          x[(size_t)(b0 + b) * N + n] = ldexpf(acc[b], -fp8_item_exponent(g.amax[b0 + b]));
        else
          x[(size_t)(b0 + b) * N + n] = acc[b];
      }
  }
}

// Block -> (tile, batch group).  XCD-aware order: workgroups are dealt
// round-robin to the 8 XCDs (each with its own L2); every XCD receives runs
// of consecutive work items (16 tiles for one batch group, else 8 tiles with
// all their groups), runs interleaved across XCDs so that the
// depth-dependent work stays balanced (the ragged last round keeps its
// order).  Work item L is batch group L mod nbg of tile L / nbg: the batch
// groups of a tile read the same sample rows (batch-inner layout), so they
// run side by side on one XCD and share those rows in its L2; a run covers
// neighbouring tiles, which stage overlapping windows.  (cfg2, 16 frames of
// four-item groups: FP32 64.4 -> 42.8 ms against batch groups outermost.)
__device__ inline void tile_of_block(int nbg, int& tile, int& bg) {
  const int X = 8, C = nbg == 1 ? 16 : 8 * nbg, per = X * C;
  const int bx = (int)blockIdx.x;
  const int L = bx >= (int)gridDim.x / per * per ? bx : bx / per * per + (bx % per % X) * C + (bx % per) / X;
  tile = L / nbg;
  bg = L - tile * nbg;
}

// Four wavefronts per SIMD (128 VGPRs) for one and two items per thread; with
// four items per thread (four accumulators, four-item tap registers and
// staging) three (168 VGPRs), which leaves no spills.
template <class T, int BT, int QN, bool WTX>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(BT >= 4 ? 3 : 4))) void tiled_forward(
    Geom g, TileShape ts, Window win, const T* __restrict__ ws, int B, float* __restrict__ x,
    int ntx, int nty, int ntiles, int nbg) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int ktx_s[16];
  __shared__ int txl_s[72];  // sparse transmit list (64) + per-wavefront masks (8)
  int tile, bg;
  tile_of_block(nbg, tile, bg);
  tile_body<T, BT, QN, WTX>(g, ts, win, ws, B, x, ntx, nty, ntiles, tile, bg * BT, smem, ktx_s,
                            txl_s);
}

// Complex baseband (IQ) variant: batch items (2b, 2b+1) are the I and Q
// records of one complex item; every term is remodulated by exp(i 2 pi fc tau)
// (the same tile schedule and windows as tiled_forward).  Three wavefronts
// per SIMD: at four it spilled 192 bytes per lane (cfg2, one complex frame:
// 8.53 -> 8.09 ms); the two-item real and the cubic kernels keep four, where
// their smaller spills cost less than the lost wavefront.
template <class T, int BT, int QN, bool WTX>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void tiled_forward_iq(
    Geom g, TileShape ts, Window win, const T* __restrict__ ws, int B, float* __restrict__ x,
    int ntx, int nty, int ntiles, int nbg) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int ktx_s[16];
  __shared__ int txl_s[72];
  int tile, bg;
  tile_of_block(nbg, tile, bg);
  tile_body<T, BT, QN, WTX, true>(g, ts, win, ws, B, x, ntx, nty, ntiles, tile, bg * BT, smem, ktx_s,
                                  txl_s);
}

// Four-point Lagrange (cubic) interpolation variant (the same tile schedule
// and windows as tiled_forward).
template <class T, int BT, int QN, bool WTX>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void tiled_forward_cubic(
    Geom g, TileShape ts, Window win, const T* __restrict__ ws, int B, float* __restrict__ x,
    int ntx, int nty, int ntiles, int nbg) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int ktx_s[16];
  __shared__ int txl_s[72];
  int tile, bg;
  tile_of_block(nbg, tile, bg);
  tile_body<T, BT, QN, WTX, false, false, true>(g, ts, win, ws, B, x, ntx, nty, ntiles, tile, bg * BT,
                                                smem, ktx_s, txl_s);
}

// Several forward passes in one persistent launch: in round r, workgroup w
// processes work item r G + ((w + 104 r) mod G) (G = gridDim.x); item i
// belongs to the plan p whose range [first[p], first[p+1]) contains it and
// names one (tile, batch group) of that plan (tiles deepest first, batch
// groups outermost).

template <class T, int BT, int QN, bool WTX>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void tiled_forward_batched(
    BatchedArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int ktx_s[16];
  __shared__ int txl_s[72];  // sparse transmit list (64) + per-wavefront masks (8)
  const int total = a.first[a.count];
  const unsigned G = gridDim.x;
  for (int r = 0; r * (int)G < total; ++r) {
    // The slot of this block rotates every round, so that it does not see the
    // same lateral tile position (and amount of work) in every round.
    const int item = r * (int)G + (int)((blockIdx.x + 104u * (unsigned)r) % G);
    if (item >= total) continue;
    int p = 0;
    while (p + 1 < a.count && item >= a.first[p + 1]) ++p;
    const PlanWork w = a.p[p];  // uniform index: copied once per item
    const int local = item - a.first[p];
    const int tile = local % w.ntiles, bg = local / w.ntiles;
    __syncthreads();  // the previous item no longer reads LDS
    tile_body<T, BT, QN, WTX, false, true>(w.g, w.ts, w.win, static_cast<const T*>(w.ws), w.B, w.x, w.ntx,
                              w.nty, w.ntiles, tile, bg * BT, smem, ktx_s, txl_s);
  }
}

template <int BT, int QN>
size_t lds_bytes_t(const Window& w) {
  return (size_t)layout(QN, chunk_elems<BT, QN>(), BT, w.pairs + 1).total;
}

template <class T, int BT, int QN, bool WTX>
hipError_t launch_t(const Geom& g, const TileShape& ts, const Window& w, const void* ws, int B,
                    float* x, hipStream_t st) {
  const int ntx = (g.n[0] + ts.tx - 1) / ts.tx, nty = (g.n[1] + ts.ty - 1) / ts.ty,
            ntz = (g.n[2] + ts.tz - 1) / ts.tz;
  const int ntiles = ntx * nty * ntz;
  const size_t lds = lds_bytes_t<BT, QN>(w);
  const int nbg = (B + BT - 1) / BT;
  dim3 grid(ntiles * nbg);
  auto kern = tiled_forward<T, BT, QN, WTX>;
  if (lds > 65536) {
    hipError_t e =
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, g, ts, w, static_cast<const T*>(ws), B, x, ntx,
                     nty, ntiles, nbg);
  return hipGetLastError();
}

// Transmit-group size for Q transmits.
inline int group_size(int Q) { return Q == 1 ? 1 : Q <= 4 ? 4 : Q <= 8 ? 8 : 16; }

template <class T, int BT, int QN, bool WTX>
hipError_t launch_iq_t(const Geom& g, const TileShape& ts, const Window& w, const void* ws, int B,
                       float* x, hipStream_t st) {
  const int ntx = (g.n[0] + ts.tx - 1) / ts.tx, nty = (g.n[1] + ts.ty - 1) / ts.ty,
            ntz = (g.n[2] + ts.tz - 1) / ts.tz;
  const int ntiles = ntx * nty * ntz;
  const size_t lds = lds_bytes_t<BT, QN>(w);
  const int nbg = (B + BT - 1) / BT;
  dim3 grid(ntiles * nbg);
  auto kern = tiled_forward_iq<T, BT, QN, WTX>;
  if (lds > 65536) {
    hipError_t e =
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, g, ts, w, static_cast<const T*>(ws), B, x, ntx,
                     nty, ntiles, nbg);
  return hipGetLastError();
}

template <class T, int BT, int QN, bool WTX>
hipError_t launch_cubic_t(const Geom& g, const TileShape& ts, const Window& w, const void* ws, int B,
                          float* x, hipStream_t st) {
  const int ntx = (g.n[0] + ts.tx - 1) / ts.tx, nty = (g.n[1] + ts.ty - 1) / ts.ty,
            ntz = (g.n[2] + ts.tz - 1) / ts.tz;
  const int ntiles = ntx * nty * ntz;
  const size_t lds = lds_bytes_t<BT, QN>(w);
  const int nbg = (B + BT - 1) / BT;
  dim3 grid(ntiles * nbg);
  auto kern = tiled_forward_cubic<T, BT, QN, WTX>;
  if (lds > 65536) {
    hipError_t e =
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, g, ts, w, static_cast<const T*>(ws), B, x, ntx,
                     nty, ntiles, nbg);
  return hipGetLastError();
}

// Cubic-interpolation launch: one, two or four items per thread as the
// linear launch.
template <class T>
hipError_t launch_cubic(const Geom& g, const TileShape& ts, const Window& w, const void* ws, int B,
                        float* x, hipStream_t st) {
  const bool wtx = g.w_tx != nullptr;
  auto pick = [&](auto bt_tag) -> hipError_t {
    constexpr int BT = decltype(bt_tag)::value;
    switch (group_size(g.Q)) {
      case 1: return wtx ? launch_cubic_t<T, BT, 1, true>(g, ts, w, ws, B, x, st)
                         : launch_cubic_t<T, BT, 1, false>(g, ts, w, ws, B, x, st);
      case 4: return wtx ? launch_cubic_t<T, BT, 4, true>(g, ts, w, ws, B, x, st)
                         : launch_cubic_t<T, BT, 4, false>(g, ts, w, ws, B, x, st);
      case 8: return wtx ? launch_cubic_t<T, BT, 8, true>(g, ts, w, ws, B, x, st)
                         : launch_cubic_t<T, BT, 8, false>(g, ts, w, ws, B, x, st);
      default: return wtx ? launch_cubic_t<T, BT, 16, true>(g, ts, w, ws, B, x, st)
                          : launch_cubic_t<T, BT, 16, false>(g, ts, w, ws, B, x, st);
    }
  };
  const int bt = tiled_batch_per_thread(DAS_STORE_F32, B);
  if (bt == 4) return pick(std::integral_constant<int, 4>());
  if (bt == 2) return pick(std::integral_constant<int, 2>());
  return pick(std::integral_constant<int, 1>());
}

// Complex baseband launch: B even (I, Q pairs), two or four items per thread.
template <class T>
hipError_t launch_iq(const Geom& g, const TileShape& ts, const Window& w, const void* ws, int B,
                     float* x, hipStream_t st) {
  const bool wtx = g.w_tx != nullptr;
  auto pick = [&](auto bt_tag) -> hipError_t {
    constexpr int BT = decltype(bt_tag)::value;
    switch (group_size(g.Q)) {
      case 1: return wtx ? launch_iq_t<T, BT, 1, true>(g, ts, w, ws, B, x, st)
                         : launch_iq_t<T, BT, 1, false>(g, ts, w, ws, B, x, st);
      case 4: return wtx ? launch_iq_t<T, BT, 4, true>(g, ts, w, ws, B, x, st)
                         : launch_iq_t<T, BT, 4, false>(g, ts, w, ws, B, x, st);
      case 8: return wtx ? launch_iq_t<T, BT, 8, true>(g, ts, w, ws, B, x, st)
                         : launch_iq_t<T, BT, 8, false>(g, ts, w, ws, B, x, st);
      default: return wtx ? launch_iq_t<T, BT, 16, true>(g, ts, w, ws, B, x, st)
                          : launch_iq_t<T, BT, 16, false>(g, ts, w, ws, B, x, st);
    }
  };
  if (B >= 4) return pick(std::integral_constant<int, 4>());
  return pick(std::integral_constant<int, 2>());
}

template <class T, int BT>
hipError_t launch_bt(const Geom& g, const TileShape& ts, const Window& w, const void* ws, int B,
                     float* x, hipStream_t st) {
  const bool wtx = g.w_tx != nullptr;
  switch (group_size(g.Q)) {
    case 1: return wtx ? launch_t<T, BT, 1, true>(g, ts, w, ws, B, x, st)
                       : launch_t<T, BT, 1, false>(g, ts, w, ws, B, x, st);
    case 4: return wtx ? launch_t<T, BT, 4, true>(g, ts, w, ws, B, x, st)
                       : launch_t<T, BT, 4, false>(g, ts, w, ws, B, x, st);
    case 8: return wtx ? launch_t<T, BT, 8, true>(g, ts, w, ws, B, x, st)
                       : launch_t<T, BT, 8, false>(g, ts, w, ws, B, x, st);
    default: return wtx ? launch_t<T, BT, 16, true>(g, ts, w, ws, B, x, st)
                        : launch_t<T, BT, 16, false>(g, ts, w, ws, B, x, st);
  }
}

inline size_t lds_bytes(int Q, int bt, const Window& w) {
  auto pick = [&](auto bt_tag) -> size_t {
    constexpr int BT = decltype(bt_tag)::value;
    switch (group_size(Q)) {
      case 1: return lds_bytes_t<BT, 1>(w);
      case 4: return lds_bytes_t<BT, 4>(w);
      case 8: return lds_bytes_t<BT, 8>(w);
      default: return lds_bytes_t<BT, 16>(w);
    }
  };
  if (bt == 4) return pick(std::integral_constant<int, 4>());
  if (bt == 2) return pick(std::integral_constant<int, 2>());
  return pick(std::integral_constant<int, 1>());
}

template <class T>
hipError_t launch(const Geom& g, const TileShape& ts, const Window& w, const void* ws, int B,
                  float* x, hipStream_t st) {
  // eight items per thread when they fill whole groups: a group then reads
  // 32 of the 64 bytes of an FP32 sample row of 16 items (four items read
  // 16, and the rest of the fetched row is waste unless another group's
  // reads hit it in L2), and the delay work is shared by twice the items
  if (B % 8 == 0) return launch_bt<T, 8>(g, ts, w, ws, B, x, st);
  const int bt = tiled_batch_per_thread(sizeof(T) == 4 ? DAS_STORE_F32 : DAS_STORE_F16, B);
  if (bt == 4) return launch_bt<T, 4>(g, ts, w, ws, B, x, st);
  if (bt == 2) return launch_bt<T, 2>(g, ts, w, ws, B, x, st);
  return launch_bt<T, 1>(g, ts, w, ws, B, x, st);
}

template <class T, int BT, int QN, bool WTX>
hipError_t launch_batched_t(const BatchedArgs& a, int cus, hipStream_t st) {
  const Window w0{0, 63};
  const size_t lds = lds_bytes_t<BT, QN>(w0);
  auto kern = tiled_forward_batched<T, BT, QN, WTX>;
  if (lds > 65536) {
    hipError_t e =
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // A persistent grid must be fully resident: a block that starts only after
  // others have finished their whole share doubles the launch time.
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, lds);
  if (e != hipSuccess) return e;
  const int grid = std::max(1, std::min(a.first[a.count], std::max(1, per_cu) * cus));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, a);
  return hipGetLastError();
}

template <class T, int BT>
hipError_t launch_batched_bt(const BatchedArgs& a, int qn, bool wtx, int cus, hipStream_t st) {
  switch (qn) {
    case 1: return wtx ? launch_batched_t<T, BT, 1, true>(a, cus, st)
                       : launch_batched_t<T, BT, 1, false>(a, cus, st);
    case 4: return wtx ? launch_batched_t<T, BT, 4, true>(a, cus, st)
                       : launch_batched_t<T, BT, 4, false>(a, cus, st);
    case 8: return wtx ? launch_batched_t<T, BT, 8, true>(a, cus, st)
                       : launch_batched_t<T, BT, 8, false>(a, cus, st);
    default: return wtx ? launch_batched_t<T, BT, 16, true>(a, cus, st)
                        : launch_batched_t<T, BT, 16, false>(a, cus, st);
  }
}

template <class T>
hipError_t launch_batched(const BatchedArgs& a, int bt, int qn, bool wtx, int cus,
                          hipStream_t st) {
  if (bt == 4) return launch_batched_bt<T, 4>(a, qn, wtx, cus, st);
  if (bt == 2) return launch_batched_bt<T, 2>(a, qn, wtx, cus, st);
  return launch_batched_bt<T, 1>(a, qn, wtx, cus, st);
}

}  // namespace tiled
}  // namespace dasmi
