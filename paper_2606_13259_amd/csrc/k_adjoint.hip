// Adjoint (scatter) and sound-speed gradient kernels, plus the delay export
// used by the delay-error test.
//
// Adjoint.  The forward map y -> x of Eq. (2) is linear; its transpose sends
// each output gradient gx[b][n] back to the two taps each (q, m) term read:
//   gy[b][q][m][k]   += w (1 - alpha) gx[b][n]
//   gy[b][q][m][k+1] += w alpha gx[b][n]      (taps inside [0, K) only).
// One workgroup owns a 256-voxel tile (the same tiles, culling and
// tile-relative delays as the windowed forward kernel).  For each chunk of
// elements it accumulates the tile's contributions in LDS windows of
// (transmit, element) channels with LDS integer atomics on fixed-point sums
// (below), then flushes every nonzero window entry to global memory with one
// float atomic.  Neighbouring
// voxels hit the same taps, so most of the scatter traffic stays in LDS.
// The windows hold 32-bit fixed-point sums: LDS integer atomics run several
// times faster than LDS float atomics on this chip.  Per (tile, transmit
// group) the largest contribution magnitude cmax is reduced over the block
// and the scale is the power of two S with cmax S < 2^22; each contribution
// is rounded to the nearest integer (absolute error <= 2^-23 cmax), a sample
// collects at most one term per voxel of the 256-voxel tile, so sums stay
// below 2^30.  The flush converts back exactly (x 1/S).  Integer sums are
// order-independent, so a tile's windows are deterministic.  The windows
// are kept in ACOPIES private copies, chosen by the voxel's x index modulo
// ACOPIES, to spread lanes that share a tap over different addresses.
// The order of the float atomics is not fixed: results are reproducible to
// FP32 rounding, not bit for bit.
//
// Sound-speed gradient.  x depends on c only through f:
//   dx/dc = sum_{q,m} w (s(k+1) - s(k)) df/dc,  df/dc = -(f + t0 fs) / c,
// (right-hand slope at integer f).  The kernel gathers like the plain forward
// kernel and reduces sum_{b,n} gx[b][n] dx[b][n]/dc to one scalar.
#include "das_device.h"

namespace dasmi {
namespace {

constexpr int QG = 16;
constexpr int NT = 256;
constexpr int MCA = 4;      // elements per adjoint chunk
constexpr int ACOPIES = 4;  // private copies of the LDS windows (power of two; cfg5: 2 copies 2.71 ms, 4 2.04 ms, 8 3.40 ms)

// Floats per window copy (a one-float pad puts the copies on different banks).
__host__ __device__ inline int copy_stride(int P) { return QG * MCA * P + 1; }

__global__ void fill_zero(float* __restrict__ p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.f;
}

hipError_t zero(float* p, size_t n, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(fill_zero, dim3((unsigned)std::max<size_t>(blocks, 1)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

struct AInfo {
  float ex, ey, ez, en, h;
  int krx, m, pad;
};

// IQ: the complex baseband form's transpose (items 2c, 2c+1 are the I and Q
// lanes of complex item c = blockIdx.y): each tap receives
// w conj(exp(i 2 pi fc tau)) times the complex upstream gradient, i.e.
// w (cos gI + sin gQ) into the I record and w (cos gQ - sin gI) into the Q
// record, with the phase of the forward (transmit and element parts in FP64,
// the tile-relative part in FP32, hardware sine and cosine on revolutions);
// two sets of windows.
template <bool IQ>
__global__ __launch_bounds__(NT) void adjoint_scatter(Geom g, TileShape ts, Window win,
                                                      const float* __restrict__ gx, int B,
                                                      float* __restrict__ gy, int ntx, int nty,
                                                      int ntiles, int per_xcd) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int P = win.pairs + 1;  // window samples
  const int cs = copy_stride(P);
  int* accw = reinterpret_cast<int*>(smem);                           // [ACOPIES][QG][MCA][P] (+pad)
  constexpr int NS = IQ ? 2 : 1;                                       // window sets (I, Q)
  AInfo* minfo = reinterpret_cast<AInfo*>(accw + NS * ACOPIES * cs);   // [MCA]
  int* ktxs = reinterpret_cast<int*>(minfo + MCA);                      // [QG]
  int* wcount = ktxs + QG;                                              // [4] (also the scale reduction)
  uint16_t* act = reinterpret_cast<uint16_t*>(wcount + 4);              // [M]

  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int tile = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (tile >= ntiles) return;
  const int b = IQ ? 2 * blockIdx.y : blockIdx.y;  // the I item for IQ
  const int tix = tile % ntx, tiy = (tile / ntx) % nty, tiz = tile / (ntx * nty);
  const int lx = t & (ts.tx - 1), ly = (t >> ts.lx) & (ts.ty - 1), lz = t >> ts.lxy;
  const int ix = tix * ts.tx + lx, iy = tiy * ts.ty + ly, iz = tiz * ts.tz + lz;
  const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
  const int K = g.K, M = g.M;

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
  const float gv = inside ? gx[(size_t)b * N + n] : 0.f;
  const float gvq = IQ && inside ? gx[(size_t)(b + 1) * N + n] : 0.f;

  const int nact = cull_elements(g, px, py, pz, hx, hy, hz, wcount, act);
  // a tile whose upstream gradient is zero everywhere scatters nothing
  if (__syncthreads_or(gv != 0.f || gvq != 0.f) == 0) return;
  // windows start at zero; every flush leaves the entries it reads at zero
  for (int i = t; i < NS * ACOPIES * cs; i += NT) accw[i] = 0;
  int* const mycopy = accw + (lx & (ACOPIES - 1)) * cs;
  int* const mycopyq = mycopy + ACOPIES * cs;  // IQ: the Q windows
  const float fcfs_f = (float)g.fcfs;

  for (int q0 = 0; q0 < g.Q; q0 += QG) {
    const int qn = min(QG, g.Q - q0);
    __syncthreads();
    if (t < qn) ktxs[t] = make_tx_ref(g, q0 + t, px, py, pz).ktx;
    float bq[QG], wq[QG];
    float wqq[IQ ? QG : 1], rq[IQ ? QG : 1];  // IQ: Q gradient and transmit phase
#pragma unroll
    for (int q = 0; q < QG; ++q) {
      bq[q] = 0.f;
      wq[q] = 0.f;
      if constexpr (IQ) wqq[q] = rq[q] = 0.f;
      if (q < qn) {
        const TxRef r = make_tx_ref(g, q0 + q, px, py, pz);
        bq[q] = fmaf(delta_tx(r, dx, dy, dz, dp2), fscf, r.g);
        const float wt = (g.w_tx && inside) ? g.w_tx[(size_t)(q0 + q) * N + n] : 1.f;
        wq[q] = gv * wt;
        if constexpr (IQ) {
          // the transmit's phase term frac(fc/fs ktx + fc t0), FP64 before rounding
          const double rv = g.fcfs * (double)r.ktx + g.fct0;
          rq[q] = (float)(rv - floor(rv));
          wqq[q] = gvq * wt;
        }
      }
    }
    // fixed-point scale of this transmit group: max |contribution| over the
    // tile (receive weights are <= 1; a rotated complex gradient is bounded
    // by |gI| + |gQ|), then S = 2^(22 - e) with cmax < 2^e
    float cm = 0.f;
#pragma unroll
    for (int q = 0; q < QG; ++q) cm = fmaxf(cm, IQ ? fabsf(wq[q]) + fabsf(wqq[IQ ? q : 0]) : fabsf(wq[q]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) cm = fmaxf(cm, __shfl_xor(cm, o));
    if (lane == 0) wcount[wave] = __float_as_int(cm);  // non-negative: int order = float order
    __syncthreads();
    const float cmax = __int_as_float(max(max(wcount[0], wcount[1]), max(wcount[2], wcount[3])));
    int e2 = 0;
    (void)frexpf(cmax, &e2);                 // cmax < 2^e2
    const float S = ldexpf(1.f, 22 - e2), invS = ldexpf(1.f, e2 - 22);
    for (int c0 = 0; c0 < nact; c0 += MCA) {
      const int mcn = min(MCA, nact - c0);
      __syncthreads();
      if (t < mcn) {
        const int m = act[c0 + t];
        const RxRef r = make_rx_ref(g, m, px, py, pz);
        minfo[t] = AInfo{r.ex, r.ey, r.ez, r.en, r.h, r.krx, m, 0};
      }
      __syncthreads();
      for (int mc = 0; mc < mcn; ++mc) {
        const AInfo mi = minfo[mc];
        const float w = rx_weight(g, mi.m, mi.ex + dx, mi.ey + dy, mi.ez + dz);
        if (__ballot(w != 0.f && (gv != 0.f || gvq != 0.f)) == 0ull) continue;
        const float a = fmaf(delta_dist(mi.ex, mi.ey, mi.ez, mi.en, dx, dy, dz, dp2), fscf, mi.h);
        int* base = mycopy + mc * P + win.dint;
        int* baseq = mycopyq + mc * P + win.dint;
        float rm = 0.f;  // IQ: the element's phase term frac(fc/fs krx)
        if constexpr (IQ) {
          const double rv = g.fcfs * (double)mi.krx;
          rm = (float)(rv - floor(rv));
        }
#pragma unroll
        for (int q = 0; q < QG; ++q) {
          if (q < qn) {
            const float f = a + bq[q];
            const float fl = floorf(f);
            const float al = f - fl;
            const int off = q * MCA * P + (int)fl;
            if constexpr (IQ) {
              // conjugate rotation: revolutions fc/fs (ktx + krx + f) + fc t0
              const float rev = frac_f32(rq[q] + rm + fcfs_f * f);
              const float sn = __builtin_amdgcn_sinf(rev), cs = __builtin_amdgcn_cosf(rev);
              const float ci = w * fmaf(cs, wq[q], sn * wqq[q]);
              const float cq = w * fmaf(cs, wqq[q], -sn * wq[q]);
              if (ci != 0.f) {
                const float cs2 = ci * S;
                atomicAdd(base + off, __float2int_rn(cs2 - cs2 * al));
                atomicAdd(base + off + 1, __float2int_rn(cs2 * al));
              }
              if (cq != 0.f) {
                const float cs2 = cq * S;
                atomicAdd(baseq + off, __float2int_rn(cs2 - cs2 * al));
                atomicAdd(baseq + off + 1, __float2int_rn(cs2 * al));
              }
            } else {
              const float c = w * wq[q];
              if (c != 0.f) {
                const float cs2 = c * S;  // exact: S is a power of two
                atomicAdd(base + off, __float2int_rn(cs2 - cs2 * al));
                atomicAdd(base + off + 1, __float2int_rn(cs2 * al));
              }
            }
          }
        }
      }
      __syncthreads();
      // flush: wave w flushes windows w, w+4, ... (IQ: then the Q windows
      // into item b + 1)
      for (int wi = wave; wi < NS * QG * MCA; wi += 4) {
        const int set = wi / (QG * MCA), q = (wi / MCA) % QG, mc = wi % MCA;
        if (q >= qn || mc >= mcn) continue;
        const int j0 = ktxs[q] + minfo[mc].krx - win.dint;
        float* dst = gy + (((size_t)(b + set) * g.Q + q0 + q) * M + minfo[mc].m) * (size_t)K;
        int* src = accw + set * ACOPIES * cs + (q * MCA + mc) * P;
        for (int p = lane; p < P; p += 64) {
          int iv = 0;
#pragma unroll
          for (int r = 0; r < ACOPIES; ++r) {
            iv += src[r * cs + p];
            src[r * cs + p] = 0;
          }
          const int j = j0 + p;
          if (iv != 0 && j >= 0 && j < K) atomicAdd(dst + j, (float)iv * invS);
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------

// One wavefront per 4 x 4 x 4 voxel box (a voxel per lane).  Elements outer,
// transmits inner, as in the forward kernels: the element's receive geometry
// and weight are formed once per (voxel, element) and reused by the transmits
// of a group of QG; elements whose receive cone misses the box's bounding
// sphere are skipped by the whole wavefront (the weight would be zero on
// every lane).
// IQ: items (2c, 2c+1) are the (I, Q) records of complex item c (BT even);
// each term also turns with the phase 2 pi fc tau, so
//   dx/dc = w exp(i 2 pi fc tau) ((s(k+1) - s(k)) + i 2 pi (fc/fs) s_interp) df/dc
// (dtau/dc = (df/dc)/fs), and the pair adds gI Re(dx/dc) + gQ Im(dx/dc).  The
// phase is formed as in the forward kernels: transmit and element parts in
// FP64 per box, the box-relative part in FP32, hardware sine and cosine.
template <int BT, bool IQ>
__global__ __launch_bounds__(256) void grad_c_gather(Geom g, const float* __restrict__ y,
                                                     const float* __restrict__ gx, int B,
                                                     float* __restrict__ out, int nbx, int nby,
                                                     int nblocks, float inv_c) {
  __shared__ float red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int blk = blockIdx.x * 4 + wave;
  const int b0 = blockIdx.y * BT;
  float total = 0.f;
  if (blk < nblocks) {
    const int bxi = blk % nbx, byi = (blk / nbx) % nby, bzi = blk / (nbx * nby);
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int ix = bxi * 4 + lx, iy = byi * 4 + ly, iz = bzi * 4 + lz;
    double px, py, pz;
    tile_ref_point(g, bxi * 4 + 1.5, byi * 4 + 1.5, bzi * 4 + 1.5, px, py, pz);
    const float dx = (float)(lx - 1.5f) * (float)g.s[0];
    const float dy = (float)(ly - 1.5f) * (float)g.s[1];
    const float dz = (float)(lz - 1.5f) * (float)g.s[2];
    const float dp2 = dx * dx + dy * dy + dz * dz;
    const float fscf = (float)g.fsc;
    const float t0fs = (float)g.t0fs;
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    const bool inside = in_grid(g, ix, iy, iz);
    const int n = grid_index(g, ix, iy, iz);
    const size_t MK = (size_t)g.M * g.K, QMK = (size_t)g.Q * MK;
    const bool hann = g.apod == DAS_APOD_HANN_FNUM;
    const float R = 1.5f * sqrtf((float)(g.s[0] * g.s[0] + g.s[1] * g.s[1] + g.s[2] * g.s[2]));
    const float tan_half = hann ? 0.5f * sqrtf(4.f / g.fourF2) : 0.f;
    float gxv[BT];
#pragma unroll
    for (int b = 0; b < BT; ++b) gxv[b] = (inside && b0 + b < B) ? gx[(size_t)(b0 + b) * N + n] : 0.f;
    const float fcfs_f = (float)g.fcfs;
    const float turn = 6.283185307179586f * fcfs_f;  // 2 pi fc / fs, radians per sample
    for (int q0 = 0; q0 < g.Q; q0 += QG) {
      const int qn = min(QG, g.Q - q0);
      float bq[QG], wq[QG];
      float rq[IQ ? QG : 1];  // IQ: the transmit's phase term (revolutions)
      int ktx[QG];
#pragma unroll
      for (int q = 0; q < QG; ++q) {
        bq[q] = 0.f;
        wq[q] = 0.f;
        ktx[q] = 0;
        if constexpr (IQ) rq[q] = 0.f;
        if (q < qn) {
          const TxRef tr = make_tx_ref(g, q0 + q, px, py, pz);
          bq[q] = fmaf(delta_tx(tr, dx, dy, dz, dp2), fscf, tr.g);
          wq[q] = (g.w_tx && inside) ? g.w_tx[(size_t)(q0 + q) * N + n] : 1.f;
          ktx[q] = tr.ktx;
          if constexpr (IQ) {
            const double rv = g.fcfs * (double)tr.ktx + g.fct0;
            rq[q] = (float)(rv - floor(rv));
          }
        }
      }
      for (int m0 = 0; m0 < g.M; m0 += 64) {
        RxRef mine = {};
        bool on = m0 + lane < g.M;
        if (on) {
          mine = make_rx_ref(g, m0 + lane, px, py, pz);
          if (hann) on = cone_hits_sphere(g, m0 + lane, px, py, pz, R, tan_half);
        }
        uint64_t mk = __ballot(on);
        while (mk) {
          const int mm = __builtin_ctzll(mk);
          mk &= mk - 1ull;
          const int m = m0 + mm;
          const float ex = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.ex), mm));
          const float ey = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.ey), mm));
          const float ez = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.ez), mm));
          const float en = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.en), mm));
          const float h = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.h), mm));
          const int krx = __builtin_amdgcn_readlane(mine.krx, mm);
          const float w = rx_weight(g, m, ex + dx, ey + dy, ez + dz);
          if (__ballot(w != 0.f) == 0ull) continue;
          const float a = fmaf(delta_dist(ex, ey, ez, en, dx, dy, dz, dp2), fscf, h);
          const float* ym = y + (size_t)q0 * MK + (size_t)m * g.K;
          float rm = 0.f;  // IQ: the element's phase term frac(fc/fs krx)
          if constexpr (IQ) {
            const double rv = g.fcfs * (double)krx;
            rm = (float)(rv - floor(rv));
          }
#pragma unroll
          for (int q = 0; q < QG; ++q) {
            if (q >= qn) break;
            const float f = a + bq[q];
            const float fl = floorf(f);
            const int kb = ktx[q] + krx;
            const int k = (int)fl + kb;
            // f + t0 fs in samples, formed in FP32 from its integer and local parts
            const float dfdc = -((float)kb + f + t0fs) * inv_c;
            const float c = w * wq[q] * dfdc;
            const float* yq = ym + (size_t)q * MK;
            if constexpr (IQ) {
              const float al = f - fl;
              const float rev = frac_f32(rq[IQ ? q : 0] + rm + fcfs_f * f);
              const float sn = __builtin_amdgcn_sinf(rev), cs = __builtin_amdgcn_cosf(rev);
#pragma unroll
              for (int b = 0; b < BT; b += 2) {
                if (b0 + b < B) {  // B even: the Q item b + 1 exists too
                  const float* yi = yq + (size_t)(b0 + b) * QMK;
                  const float* yqq = yi + QMK;
                  const bool in1 = k >= 0 && k < g.K, in2 = k + 1 >= 0 && k + 1 < g.K;
                  const float i1 = in1 ? yi[k] : 0.f, i2 = in2 ? yi[k + 1] : 0.f;
                  const float q1 = in1 ? yqq[k] : 0.f, q2 = in2 ? yqq[k + 1] : 0.f;
                  const float di = i2 - i1, dq = q2 - q1;
                  const float vi = fmaf(al, di, i1), vq = fmaf(al, dq, q1);
                  const float zi = fmaf(-turn, vq, di), zq = fmaf(turn, vi, dq);
                  const float ri = fmaf(cs, zi, -sn * zq), rqv = fmaf(sn, zi, cs * zq);
                  total = fmaf(c, fmaf(gxv[b], ri, gxv[b + 1] * rqv), total);
                }
              }
            } else {
#pragma unroll
              for (int b = 0; b < BT; ++b) {
                if (b0 + b < B) {
                  const float* yb = yq + (size_t)(b0 + b) * QMK;
                  const float s1 = (k >= 0 && k < g.K) ? yb[k] : 0.f;
                  const float s2 = (k + 1 >= 0 && k + 1 < g.K) ? yb[k + 1] : 0.f;
                  total = fmaf(gxv[b] * c, s2 - s1, total);
                }
              }
            }
          }
        }
      }
    }
  }
  // wave + block reduction, one atomic per block
  for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off);
  if (lane == 0) red[wave] = total;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, red[0] + red[1] + red[2] + red[3]);
}

// ----------------------------------------------------------------------------

__global__ void debug_delays(Geom g, TileShape ts, int q, int m0, int m1, int n0, int n1,
                             double* __restrict__ out) {
  const long long nn = n1 - n0;
  const long long total = (long long)(m1 - m0) * nn;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int m = m0 + (int)(i / nn);
  const int n = n0 + (int)(i % nn);
  const int ix = n % g.n[0], iy = (n / g.n[0]) % g.n[1], iz = n / (g.n[0] * g.n[1]);
  const int tix = ix / ts.tx, tiy = iy / ts.ty, tiz = iz / ts.tz;
  const float hx = 0.5f * (ts.tx - 1), hy = 0.5f * (ts.ty - 1), hz = 0.5f * (ts.tz - 1);
  double px, py, pz;
  tile_ref_point(g, tix * ts.tx + (double)hx, tiy * ts.ty + (double)hy, tiz * ts.tz + (double)hz,
                 px, py, pz);
  const float dx = ((float)(ix - tix * ts.tx) - hx) * (float)g.s[0];
  const float dy = ((float)(iy - tiy * ts.ty) - hy) * (float)g.s[1];
  const float dz = ((float)(iz - tiz * ts.tz) - hz) * (float)g.s[2];
  const float dp2 = dx * dx + dy * dy + dz * dz;
  const float fscf = (float)g.fsc;
  const RxRef r = make_rx_ref(g, m, px, py, pz);
  const TxRef tr = make_tx_ref(g, q, px, py, pz);
  const float a = fmaf(delta_dist(r.ex, r.ey, r.ez, r.en, dx, dy, dz, dp2), fscf, r.h);
  const float bq = fmaf(delta_tx(tr, dx, dy, dz, dp2), fscf, tr.g);
  out[i] = (double)(r.krx + tr.ktx) + (double)(a + bq);
}

}  // namespace

size_t adjoint_lds_bytes(const Geom& g, const Window& w) {
  const int P = w.pairs + 1;
  size_t lds = (size_t)(g.iq ? 2 : 1) * ACOPIES * copy_stride(P) * 4 + MCA * sizeof(AInfo) + QG * 4 + 16 +
               (size_t)g.M * 2;
  return (lds + 15) & ~(size_t)15;
}

hipError_t launch_adjoint(const Geom& g, const TileShape& ts, const Window& w, const float* gx,
                          int B, float* gy, hipStream_t st) {
  hipError_t e = zero(gy, (size_t)B * g.Q * g.M * g.K, st);
  if (e != hipSuccess) return e;
  const int ntx = (g.n[0] + ts.tx - 1) / ts.tx, nty = (g.n[1] + ts.ty - 1) / ts.ty,
            ntz = (g.n[2] + ts.tz - 1) / ts.tz;
  const int ntiles = ntx * nty * ntz;
  const int per_xcd = (ntiles + 7) / 8;
  const size_t lds = adjoint_lds_bytes(g, w);
  // complex baseband: one workgroup per (I, Q) item pair
  const void* kern = g.iq ? (const void*)adjoint_scatter<true> : (const void*)adjoint_scatter<false>;
  if (lds > 65536) {
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (g.iq)
    hipLaunchKernelGGL(adjoint_scatter<true>, dim3(per_xcd * 8, B / 2), dim3(NT), lds, st, g, ts, w,
                       gx, B, gy, ntx, nty, ntiles, per_xcd);
  else
    hipLaunchKernelGGL(adjoint_scatter<false>, dim3(per_xcd * 8, B), dim3(NT), lds, st, g, ts, w,
                       gx, B, gy, ntx, nty, ntiles, per_xcd);
  return hipGetLastError();
}

hipError_t launch_grad_c(const Geom& g, const float* y, const float* gx, int B, float* dLdc,
                         hipStream_t st) {
  hipError_t e = zero(dLdc, 1, st);
  if (e != hipSuccess) return e;
  const int nbx = (g.n[0] + 3) / 4, nby = (g.n[1] + 3) / 4, nbz = (g.n[2] + 3) / 4;
  const int nblocks = nbx * nby * nbz;
  const float inv_c = (float)(1.0 / g.c);
  if (g.iq) {  // B even: pairs never straddle a block (BT even)
    if (B >= 4)
      hipLaunchKernelGGL((grad_c_gather<4, true>), dim3((nblocks + 3) / 4, (B + 3) / 4), dim3(256), 0,
                         st, g, y, gx, B, dLdc, nbx, nby, nblocks, inv_c);
    else
      hipLaunchKernelGGL((grad_c_gather<2, true>), dim3((nblocks + 3) / 4, (B + 1) / 2), dim3(256), 0,
                         st, g, y, gx, B, dLdc, nbx, nby, nblocks, inv_c);
  } else if (B >= 4) {
    hipLaunchKernelGGL((grad_c_gather<4, false>), dim3((nblocks + 3) / 4, (B + 3) / 4), dim3(256), 0,
                       st, g, y, gx, B, dLdc, nbx, nby, nblocks, inv_c);
  } else if (B >= 2) {
    hipLaunchKernelGGL((grad_c_gather<2, false>), dim3((nblocks + 3) / 4, (B + 1) / 2), dim3(256), 0,
                       st, g, y, gx, B, dLdc, nbx, nby, nblocks, inv_c);
  } else {
    hipLaunchKernelGGL((grad_c_gather<1, false>), dim3((nblocks + 3) / 4, B), dim3(256), 0, st, g, y,
                       gx, B, dLdc, nbx, nby, nblocks, inv_c);
  }
  return hipGetLastError();
}

hipError_t launch_debug_delays(const Geom& g, const TileShape& ts, int q, int m0, int m1, int n0,
                               int n1, double* f_out, hipStream_t st) {
  const long long total = (long long)(m1 - m0) * (n1 - n0);
  const unsigned blocks = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(debug_delays, dim3(blocks), dim3(256), 0, st, g, ts, q, m0, m1, n0, n1, f_out);
  return hipGetLastError();
}

}  // namespace dasmi
