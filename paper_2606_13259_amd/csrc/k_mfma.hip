// Matrix-core (MFMA) locality form of the forward pass: the tensor-core
// method of Sec. 3.4 (Alg. 3), re-designed around gfx950's
// v_mfma_f32_16x16x32_{f16,bf16}.
//
// Neighbouring voxels take their taps from nearly the same samples of each
// channel (Sec. 3.1, 3.4), so for a group of 16 voxels the sparse gather
// turns into a dense product X += W Y:
//   * rows (16): the voxels of a 4x4x1 group (lateral, one depth: the delay
//     changes least across it);
//   * contraction (32) = 4 receivers x 8 consecutive samples (one "chunk");
//   * columns (16 per MFMA, NB MFMAs per wavefront): batch items.
// Lane l of a wavefront owns voxel l%16 and receiver row l/16.  W[n][(r, s)]
// holds w(1 - alpha) and w alpha at the voxel's tap k and k+1 when they fall
// in chunk s of receiver r, zero elsewhere.  Each receiver row covers the
// chunks between the smallest and largest tap of its 16 voxels (a DPP min/max
// over the row: the paper's per-receiver set of unique sample indices, kept
// contiguous), so the number of MFMAs per (receiver quad, transmit) follows
// the actual tap spread.  Receivers whose receive cone misses the whole group
// are culled first (conservative sphere-cone test), and quads are formed from
// the surviving receivers.
//
// Workspace ("chunked batch-inner"): ws[q][m][kc][Bp][8] in f16 or bf16, chunk
// kc holding samples 8 (kc - 1) .. 8 kc - 1 (zero outside [0, K)), Kc =
// ceil(K/8) + 2 chunks, Bp = batch rounded up to 16.  The B fragment of a
// lane (batch item b, receiver row r) is one 16-byte load, and the 16 lanes of
// a row read 256 contiguous bytes.
//
// Delay formation is the tile-relative FP32 scheme of the VALU kernels with
// the group centre as reference.  Weights are rounded to the operand type;
// for bf16 each weight is split into a high and a low bf16 part (two MFMAs
// with the same samples) so that the weight rounding stays far below the
// storage rounding.  Accumulation is FP32.
#include "das_device.h"

namespace dasmi {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf168 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int CH = 8;  // samples per chunk

__device__ inline uint16_t f16_bits(float v) {
  const _Float16 h = (_Float16)v;
  return __builtin_bit_cast(uint16_t, h);
}
// float -> bf16 bits, round to nearest even, NaN kept quiet.
__device__ inline uint16_t bf16_bits(float v) {
  const uint32_t u = __float_as_uint(v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_value(float v) { return __uint_as_float((uint32_t)bf16_bits(v) << 16); }

template <class T> struct Mma;
template <> struct Mma<_Float16> {
  static constexpr bool kSplit = false;
  __device__ static f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8, a),
                                                   __builtin_bit_cast(half8, b), c, 0, 0, 0);
  }
  __device__ static uint32_t pack(float a, float b) {
    return (uint32_t)f16_bits(a) | ((uint32_t)f16_bits(b) << 16);
  }
};
template <> struct Mma<uint16_t> {  // bf16 bit patterns
  static constexpr bool kSplit = true;
  __device__ static f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf168, a),
                                                    __builtin_bit_cast(bf168, b), c, 0, 0, 0);
  }
  __device__ static uint32_t pack(float a, float b) {
    return (uint32_t)bf16_bits(a) | ((uint32_t)bf16_bits(b) << 16);
  }
};

// Put the packed pair P = (w1, w2) at 16-bit slots (d, d+1) of an 8-slot
// fragment; slots outside [0, 8) are dropped.
__device__ inline u32x4 place_pair(uint32_t P, int d) {
  const uint64_t x = P;
  const int d1 = d - 4;
  const uint64_t lo = ((unsigned)d <= 3u) ? (x << ((16 * d) & 63)) : (d == -1 ? (x >> 16) : 0ull);
  const uint64_t hi = ((unsigned)d1 <= 3u) ? (x << ((16 * d1) & 63)) : (d1 == -1 ? (x >> 16) : 0ull);
  return u32x4{(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
}

// Min / max over the 16 lanes of a DPP row (rotations by 1, 2, 4, 8).
__device__ inline int row_min(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x121, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x122, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x124, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x128, 0xf, 0xf, false));
  return v;
}
__device__ inline int row_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x121, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x122, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x124, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x128, 0xf, 0xf, false));
  return v;
}

// Can any point of the sphere (centre p0, radius R) lie in the receive cone of
// the element (e = p0 - r_m, axis n, half-angle with cos cth, sin sth)?
// Conservative and trig-free: cos(phi) > cos(theta + beta).
__device__ inline bool sphere_in_cone(float ex, float ey, float ez, float nx, float ny, float nz,
                                      float R, float cth, float sth) {
  const float D2 = ex * ex + ey * ey + ez * ez;
  if (D2 <= R * R * 1.0001f) return true;
  const float invD = __builtin_amdgcn_rsqf(D2);
  const float cphi = (ex * nx + ey * ny + ez * nz) * invD;
  const float sb = R * invD;
  const float cb = __builtin_amdgcn_sqrtf(fmaxf(0.f, 1.f - sb * sb));
  return cphi > cth * cb - sth * sb - 1e-4f;
}

template <class T, int NB, int QN, bool WTX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void mfma_forward(
    Geom g, const T* __restrict__ ws, int B,
                                                    int Bp, int Kc, float* __restrict__ x, int ngx,
                                                    int ngy, int ngroups) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = blockIdx.x * 4 + wave;
  if (grp >= ngroups) return;  // whole wavefront
  // deepest groups first (they see the most receivers)
  const int per_z = ngx * ngy;
  const int gz = g.n[2] - 1 - grp / per_z;
  const int gx = grp % ngx, gy = (grp / ngx) % ngy;
  const int vi = lane & 15, row = lane >> 4;
  const int ix = gx * 4 + (vi & 3), iy = gy * 4 + (vi >> 2);
  const int b0 = blockIdx.y * 16 * NB;
  const int M = g.M, K = g.K;
  const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];

  double px, py, pz;
  tile_ref_point(g, gx * 4 + 1.5, gy * 4 + 1.5, (double)gz, px, py, pz);
  const float sx = (float)g.s[0], sy = (float)g.s[1];
  const float dx = ((float)(vi & 3) - 1.5f) * sx, dy = ((float)(vi >> 2) - 1.5f) * sy, dz = 0.f;
  const float dp2 = dx * dx + dy * dy;
  const float fscf = (float)g.fsc;
  const bool inside = in_grid(g, ix, iy, gz);
  const int n = inside ? grid_index(g, ix, iy, gz) : 0;
  const float Rg = 1.5f * sqrtf(sx * sx + sy * sy);
  const bool hann = g.apod == DAS_APOD_HANN_FNUM;
  const float cth = hann ? sqrtf(g.fourF2) * rsqrtf(1.f + g.fourF2) : -1.f;
  const float sth = hann ? rsqrtf(1.f + g.fourF2) : 0.f;
  const size_t chunk_stride = (size_t)Bp * CH;  // elements per chunk
  const size_t chan_stride = (size_t)Kc * chunk_stride;
  const int nbv = min(NB, (Bp - b0) >> 4);       // batch tiles present (uniform)
  constexpr int BIG = 1 << 29;

  f32x4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int q0 = 0; q0 < g.Q; q0 += QN) {
    const int qn = min(QN, g.Q - q0);
    TxRef mine = {};
    if (lane < qn) mine = make_tx_ref(g, q0 + lane, px, py, pz);
    float bq[QN], wq[WTX ? QN : 1];
    int ktx[QN];
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      TxRef r;
      r.kind = __shfl(mine.kind, q);
      r.vx = __shfl(mine.vx, q);
      r.vy = __shfl(mine.vy, q);
      r.vz = __shfl(mine.vz, q);
      r.vn = __shfl(mine.vn, q);
      ktx[q] = __builtin_amdgcn_readfirstlane(__shfl(mine.ktx, q));
      bq[q] = fmaf(delta_tx(r, dx, dy, dz, dp2), fscf, __shfl(mine.g, q));
      if constexpr (WTX) wq[q] = (q < qn && inside) ? g.w_tx[(size_t)(q0 + q) * N + n] : 0.f;
    }
    for (int m0 = 0; m0 < M; m0 += 64) {
      // one receiver per lane: group-level cone test and FP64 reference terms
      const int me = m0 + lane;
      bool on = me < M;
      float rex = 0.f, rey = 0.f, rez = 0.f, ren = 0.f, rh = 0.f;
      int rk = 0;
      if (on) {
        const double ex = px - g.elem[3 * me + 0];
        const double ey = py - g.elem[3 * me + 1];
        const double ez = pz - g.elem[3 * me + 2];
        rex = (float)ex;
        rey = (float)ey;
        rez = (float)ez;
        if (hann) {
          float nx = 0.f, ny = 0.f, nz = 1.f;
          if (g.enorm) {
            nx = g.enorm[3 * me + 0];
            ny = g.enorm[3 * me + 1];
            nz = g.enorm[3 * me + 2];
          }
          on = sphere_in_cone(rex, rey, rez, nx, ny, nz, Rg, cth, sth);
        }
        if (on) {
          const double R = sqrt(ex * ex + ey * ey + ez * ez);
          const double fr = R * g.fsc;
          const double fl = floor(fr);
          ren = (float)R;
          rh = (float)(fr - fl);
          rk = (int)fl;
        }
      }
      uint64_t mk = __ballot(on);
      while (mk) {
        // next (up to) four surviving receivers, one per row
        int js[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          js[r] = mk ? __builtin_ctzll(mk) : -1;
          mk &= mk - 1ull;
        }
        const int j = row == 0 ? js[0] : row == 1 ? js[1] : row == 2 ? js[2] : js[3];
        const int src = j < 0 ? 0 : j;
        const float ex = __shfl(rex, src), ey = __shfl(rey, src), ez = __shfl(rez, src);
        const float en = __shfl(ren, src), h = __shfl(rh, src);
        const int krx = __shfl(rk, src);
        const int m = m0 + src;
        const float w = j < 0 ? 0.f : rx_weight(g, m, ex + dx, ey + dy, ez + dz);
        if (__ballot(w != 0.f) == 0ull) continue;
        const float a = fmaf(delta_dist(ex, ey, ez, en, dx, dy, dz, dp2), fscf, h);
        const T* chan = ws + ((size_t)q0 * M + m) * chan_stride + (size_t)(b0 + vi) * CH;
#pragma unroll
        for (int q = 0; q < QN; ++q) {
          if (q >= qn) break;  // uniform
          const float f = a + bq[q];
          const int t = ktx[q] + krx + floor_i32(f);  // absolute tap index
          const float al = frac_f32(f);
          // taps outside [-1, K-1] read only zero padding
          const bool valid = w != 0.f && t >= -1 && t <= K - 1;
          const float wt = valid ? (WTX ? w * wq[WTX ? q : 0] : w) : 0.f;
          const float w2 = wt * al, w1 = wt - w2;
          const uint32_t P = Mma<T>::pack(w1, w2);
          uint32_t Plo = 0;
          if constexpr (Mma<T>::kSplit) Plo = Mma<T>::pack(w1 - bf16_value(w1), w2 - bf16_value(w2));
          // chunk range of this receiver row: samples [tmin, tmax + 1]
          const int tmin = row_min(valid ? t : BIG);
          const int tmax = row_max(valid ? t : -BIG);
          const int c_lo = (tmin + CH) >> 3;  // chunk holding sample tmin
          const int nrow = tmax < tmin ? 0 : ((tmax + 1 + CH) >> 3) - c_lo + 1;
          const int nc = max(max(__builtin_amdgcn_readlane(nrow, 0), __builtin_amdgcn_readlane(nrow, 16)),
                             max(__builtin_amdgcn_readlane(nrow, 32), __builtin_amdgcn_readlane(nrow, 48)));
          const T* cq = chan + (size_t)q * M * chan_stride;
          const int dv = valid ? t + CH - CH * c_lo : -BIG;  // slot of tap t in chunk c_lo
          // Nearly every row spans one or two chunks: issue both chunks' loads
          // unconditionally (clamped addresses, zero weights when unused),
          // then the MFMAs, then any further chunks.
          {
            const T* p0 = cq + (size_t)min(max(c_lo, 0), Kc - 1) * chunk_stride;
            const T* p1 = cq + (size_t)min(max(c_lo + 1, 0), Kc - 1) * chunk_stride;
            u32x4 B0[NB], B1[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
              if (nb < nbv) {
                B0[nb] = *reinterpret_cast<const u32x4*>(p0 + nb * 16 * CH);
                B1[nb] = *reinterpret_cast<const u32x4*>(p1 + nb * 16 * CH);
              }
            }
            const u32x4 A0 = place_pair(P, dv), A1 = place_pair(P, dv - CH);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
              if (nb < nbv) {
                acc[nb] = Mma<T>::mma(A0, B0[nb], acc[nb]);
                acc[nb] = Mma<T>::mma(A1, B1[nb], acc[nb]);
              }
            }
            if constexpr (Mma<T>::kSplit) {
              const u32x4 L0 = place_pair(Plo, dv), L1 = place_pair(Plo, dv - CH);
#pragma unroll
              for (int nb = 0; nb < NB; ++nb) {
                if (nb < nbv) {
                  acc[nb] = Mma<T>::mma(L0, B0[nb], acc[nb]);
                  acc[nb] = Mma<T>::mma(L1, B1[nb], acc[nb]);
                }
              }
            }
          }
          for (int u = 2; u < nc; ++u) {
            const int cc = min(max(c_lo + u, 0), Kc - 1);
            const T* p = cq + (size_t)cc * chunk_stride;
            const int d = dv - CH * u;
            const u32x4 A = place_pair(P, d);
            u32x4 Bf[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              if (nb < nbv) Bf[nb] = *reinterpret_cast<const u32x4*>(p + nb * 16 * CH);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              if (nb < nbv) acc[nb] = Mma<T>::mma(A, Bf[nb], acc[nb]);
            if constexpr (Mma<T>::kSplit) {
              const u32x4 Al = place_pair(Plo, d);
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
                if (nb < nbv) acc[nb] = Mma<T>::mma(Al, Bf[nb], acc[nb]);
            }
          }
        }
      }
    }
  }
  // result: lane holds batch column vi and voxel rows 4 row + r (x = r, y = row)
  const int jy = gy * 4 + row;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int b = b0 + nb * 16 + vi;
    if (nb >= nbv || b >= B || jy >= g.n[1]) continue;
    float* xb = x + (size_t)b * N + (size_t)g.n[0] * (jy + (size_t)g.n[1] * gz);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jx = gx * 4 + r;
      if (jx < g.n[0]) xb[jx] = acc[nb][r];
    }
  }
}

// y[nb][Q][M][K] f32 -> chunked batch-inner ws[Q][M][Kc][Bp][8] for items
// b0 .. b0+nb-1.  A workgroup converts 32 chunks (256 samples) of 16 items of
// one channel (q, m): rows of 256 samples are read coalesced into LDS, then
// each thread packs two 8-sample chunks, the 16 items of a chunk being
// adjacent 16-byte stores.
constexpr int RC = 32;  // chunks per reorder tile
template <class T>
__global__ __launch_bounds__(256) void reorder_chunks(const float* __restrict__ y, int Q, int M,
                                                      int K, int Kc, int nb, int b0, int Bp,
                                                      T* __restrict__ ws) {
  __shared__ float tile[16][RC * CH + 1];
  const long long QM = (long long)Q * M;
  const int t = threadIdx.x;
  const int kc0 = blockIdx.x * RC;
  const int i0 = blockIdx.z * 16;  // first item of this tile (relative to b0)
  for (long long qm = blockIdx.y; qm < QM; qm += gridDim.y) {
    const int k = CH * (kc0 - 1) + t;
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
      const int b = i0 + i;
      tile[i][t] = (b < nb && k >= 0 && k < K) ? y[((long long)b * QM + qm) * K + k] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int o = t + 256 * j;
      const int kcl = o >> 4, i = o & 15;
      const int kc = kc0 + kcl, b = i0 + i;
      if (kc < Kc && b < nb) {
        uint32_t v[CH];
#pragma unroll
        for (int s = 0; s < CH; ++s) {
          const float f = tile[i][kcl * CH + s];
          if constexpr (__is_same(T, _Float16))
            v[s] = f16_bits(f);
          else
            v[s] = bf16_bits(f);
        }
        const u32x4 o4{v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16),
                       v[6] | (v[7] << 16)};
        *reinterpret_cast<u32x4*>(ws + ((qm * Kc + kc) * Bp + b0 + b) * CH) = o4;
      }
    }
    __syncthreads();
  }
}

template <class T, int NB, int QN, bool WTX>
hipError_t launch_t(const Geom& g, const void* ws, int B, float* x, hipStream_t st) {
  const int ngx = (g.n[0] + 3) / 4, ngy = (g.n[1] + 3) / 4;
  const int ngroups = ngx * ngy * g.n[2];
  const int Bp = mfma_batch_pad(B), Kc = mfma_chunks(g.K);
  dim3 grid((ngroups + 3) / 4, (Bp + 16 * NB - 1) / (16 * NB));
  hipLaunchKernelGGL((mfma_forward<T, NB, QN, WTX>), grid, dim3(256), 0, st, g,
                     static_cast<const T*>(ws), B, Bp, Kc, x, ngx, ngy, ngroups);
  return hipGetLastError();
}

template <class T, int NB>
hipError_t launch_nb(const Geom& g, const void* ws, int B, float* x, hipStream_t st) {
  const bool wtx = g.w_tx != nullptr;
  const int qg = g.Q == 1 ? 1 : g.Q <= 4 ? 4 : g.Q <= 8 ? 8 : 16;
  switch (qg) {
    case 1: return wtx ? launch_t<T, NB, 1, true>(g, ws, B, x, st) : launch_t<T, NB, 1, false>(g, ws, B, x, st);
    case 4: return wtx ? launch_t<T, NB, 4, true>(g, ws, B, x, st) : launch_t<T, NB, 4, false>(g, ws, B, x, st);
    case 8: return wtx ? launch_t<T, NB, 8, true>(g, ws, B, x, st) : launch_t<T, NB, 8, false>(g, ws, B, x, st);
    default: return wtx ? launch_t<T, NB, 16, true>(g, ws, B, x, st) : launch_t<T, NB, 16, false>(g, ws, B, x, st);
  }
}

template <class T>
hipError_t launch_any(const Geom& g, const void* ws, int B, float* x, hipStream_t st) {
  if (B > 32) return launch_nb<T, 4>(g, ws, B, x, st);
  if (B > 16) return launch_nb<T, 2>(g, ws, B, x, st);
  return launch_nb<T, 1>(g, ws, B, x, st);
}

}  // namespace

int mfma_batch_pad(int B) { return (B + 15) & ~15; }
int mfma_chunks(int K) { return (K + CH - 1) / CH + 2; }

size_t mfma_workspace_elems(const Geom& g, int B) {
  return (size_t)g.Q * g.M * mfma_chunks(g.K) * mfma_batch_pad(B) * CH;
}

hipError_t launch_mfma_reorder(const Geom& g, int storage, const float* y, int b0, int nb, int btot,
                               void* ws, hipStream_t st) {
  const int Kc = mfma_chunks(g.K), Bp = mfma_batch_pad(btot);
  const long long QM = (long long)g.Q * g.M;
  const dim3 grid((Kc + RC - 1) / RC, (unsigned)std::min<long long>(QM, 65535), (nb + 15) / 16);
  if (storage == DAS_STORE_F16)
    hipLaunchKernelGGL(reorder_chunks<_Float16>, grid, dim3(256), 0, st, y, g.Q, g.M, g.K, Kc, nb,
                       b0, Bp, static_cast<_Float16*>(ws));
  else
    hipLaunchKernelGGL(reorder_chunks<uint16_t>, grid, dim3(256), 0, st, y, g.Q, g.M, g.K, Kc, nb,
                       b0, Bp, static_cast<uint16_t*>(ws));
  return hipGetLastError();
}

hipError_t launch_mfma_forward(const Geom& g, int storage, const void* ws, int B, float* x,
                               hipStream_t st) {
  if (storage == DAS_STORE_F16) return launch_any<_Float16>(g, ws, B, x, st);
  return launch_any<uint16_t>(g, ws, B, x, st);
}

}  // namespace dasmi
