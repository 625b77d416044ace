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
// Workspace ("batch-tiled chunks"): ws[Bp/TW][q][m][kc][TW][8] in f16, bf16 or FP8,
// chunk kc holding samples 8 (kc - 1) .. 8 kc - 1 (zero outside [0, K)),
// Kc = ceil(K/8) + 2 chunks, TW = 16 NB batch items per tile (NB = 1, 2, 4 by
// batch size) and Bp the batch rounded up to TW.  The B fragment of a lane
// (batch item b, receiver row r) is one 16-byte load (8 bytes for FP8), the
// 16 lanes of a row read 256 (128) contiguous bytes, and the wavefronts of one
// batch tile sweep one contiguous region.  FP8 (E4M3) codes are decoded to f16
// operands in registers, exactly, or (FP8-operand forms) contracted as they
// are by the FP8 matrix instructions; the item's power-of-two scale is
// removed at the output.
//
// A wavefront owns a box of four such groups, a 4 x 4 x 4 column (groups
// stacked in depth) or an 8 x 8 x 1 slab (groups side by side): it loads the
// union of their chunks once per receiver row and applies each loaded chunk
// to every group of the box with taps in it, which divides the L1/L2
// traffic by up to four.
//
// Delay formation is the tile-relative FP32 scheme of the VALU kernels with
// the box centre as reference.  Weights are rounded to the operand type; for
// bf16 and FP8 operands each weight is split into a high and a low part (two
// MFMAs with the same samples) so that the weight rounding stays below the
// storage rounding.  Accumulation is FP32.
#include "mfma_common.h"

namespace dasmi {
namespace {

using namespace mfma;

// Box form: one wavefront owns a box of ZS = GX GY GZ voxel groups (GX x GY
// lateral groups of 4 x 4 voxels, GZ depths) for 16 NB batch columns.  Per
// receiver row it loads the union of the groups' chunks once, and applies to
// each loaded chunk the A fragments of the groups that have taps in it (a
// wave-uniform test per (group, chunk)), so a chunk read from L2 serves up to
// ZS groups: lateral neighbours at one depth take their taps from nearly the
// same samples, depth neighbours from samples about half a chunk apart per
// voxel.  Delays are formed relative to the box centre.  The per-transmit
// delay terms (and transmit weights) of a group of QN transmits live in LDS
// (bq_lds: QN x 64 lanes x ZS floats per wavefront, each lane reading only its
// own entries), which keeps them out of the register budget of the chunk loop.
template <int X, int Y, int Z>
struct Box {
  static constexpr int GX = X, GY = Y, GZ = Z, ZS = X * Y * Z;
};

// IQ: complex baseband items come in (I, Q) column pairs; every term is
// remodulated by exp(i 2 pi fc tau).  Two accumulators take the same sample
// fragments with the weights times cos and times sin of the phase; since the
// sum is linear, I = acc_cos(I) - acc_sin(Q) and Q = acc_sin(I) + acc_cos(Q)
// are combined once at the end (one lane exchange: columns 2c and 2c+1 are
// neighbouring lanes).
template <class S, class BX, int NB, int QN, bool WTX, class OP = Operand<S>, bool IQ = false>
__device__ __forceinline__ void stack_body(const Geom& g, const S* __restrict__ ws, int B, int TW,
                                           int Kc, float* __restrict__ x, int ngx, int ngy,
                                           int col, int by, float* __restrict__ bq_lds) {
  using T = typename OP::T;
  constexpr int GX = BX::GX, GY = BX::GY, GZ = BX::GZ, ZS = BX::ZS;
  // chunks loaded per step before the rare second pass
  constexpr int NCH = GZ == 1 ? 3 : GZ / 2 + 2;
  const int lane = threadIdx.x & 63;
  const int per_z = ngx * ngy;
  const int gz0 = g.n[2] - GZ * (col / per_z + 1);  // first depth of the box (deepest first)
  const int bx0 = (col % ngx) * 4 * GX, by0 = ((col / ngx) % ngy) * 4 * GY;  // first voxel
  const int vi = lane & 15, row = lane >> 4;
  const int M = g.M, K = g.K;
  const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
  const int subs = TW / (16 * NB);
  const int tile = by / subs, col0 = (by - tile * subs) * 16 * NB;

  const float hx = 0.5f * (4 * GX - 1), hy = 0.5f * (4 * GY - 1), hzv = 0.5f * (GZ - 1);
  double px, py, pz;
  tile_ref_point(g, bx0 + (double)hx, by0 + (double)hy, gz0 + (double)hzv, px, py, pz);
  const float sx = (float)g.s[0], sy = (float)g.s[1], sz = (float)g.s[2];
  float dx[ZS], dy[ZS], dz[ZS], dp2[ZS];
  int nk[ZS];
  bool ink[ZS];
#pragma unroll
  for (int k = 0; k < ZS; ++k) {
    const int kx = k % GX, ky = (k / GX) % GY, kz = k / (GX * GY);
    const int lx = 4 * kx + (vi & 3), ly = 4 * ky + (vi >> 2);
    dx[k] = ((float)lx - hx) * sx;
    dy[k] = ((float)ly - hy) * sy;
    dz[k] = ((float)kz - hzv) * sz;
    dp2[k] = dx[k] * dx[k] + dy[k] * dy[k] + dz[k] * dz[k];
    ink[k] = bx0 + lx < g.n[0] && by0 + ly < g.n[1] && gz0 + kz >= 0;
    nk[k] = ink[k] ? grid_index(g, bx0 + lx, by0 + ly, gz0 + kz) : 0;
  }
  const float fscf = (float)g.fsc;
  const float Rg = sqrtf(hx * hx * sx * sx + hy * hy * sy * sy + hzv * hzv * sz * sz);
  const bool hann = g.apod == DAS_APOD_HANN_FNUM;
  const float cth = hann ? sqrtf(g.fourF2) * rsqrtf(1.f + g.fourF2) : -1.f;
  const float sth = hann ? rsqrtf(1.f + g.fourF2) : 0.f;
  const uint32_t chunk_el = (uint32_t)TW * CH;
  const size_t chan_el = (size_t)Kc * chunk_el;
  const size_t q_el = (size_t)M * chan_el;
  const S* wtile = ws + (size_t)tile * g.Q * q_el + (size_t)(col0 + vi) * CH;
  constexpr int BIG = 1 << 29;

  f32x4 acc[ZS][NB];
  f32x4 acs[IQ ? ZS : 1][IQ ? NB : 1];  // IQ: sine-weighted accumulators
#pragma unroll
  for (int k = 0; k < ZS; ++k)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      acc[k][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
      if constexpr (IQ) acs[k][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  const float fcfs_f = (float)g.fcfs;

  for (int q0 = 0; q0 < g.Q; q0 += QN) {
    const int qn = min(QN, g.Q - q0);
    TxRef mine = {};
    if (lane < qn) mine = make_tx_ref(g, q0 + lane, px, py, pz);
    // per (transmit, lane): ZS delay terms and, with transmit weights, ZS weights
    constexpr int PER = WTX ? 2 * ZS : ZS;
    float* bql = bq_lds + (size_t)(threadIdx.x >> 6) * QN * 64 * PER + lane * PER;
    const int my_ktx = mine.ktx;
    // IQ: the transmit's phase term frac(fc/fs ktx + fc t0) in revolutions
    // (FP64 before rounding: ktx reaches thousands)
    float my_rq = 0.f;
    if constexpr (IQ) {
      const double rv = g.fcfs * (double)my_ktx + g.fct0;
      my_rq = (float)(rv - floor(rv));
    }
    // transmits of the group with a nonzero weight somewhere in this column
    // (sparse transmit lists, Sec. 5: the others contribute exact zeros)
    uint32_t qact = (1u << qn) - 1u;
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      TxRef r;
      r.kind = __shfl(mine.kind, q);
      r.vx = __shfl(mine.vx, q);
      r.vy = __shfl(mine.vy, q);
      r.vz = __shfl(mine.vz, q);
      r.vn = __shfl(mine.vn, q);
      const float gq = __shfl(mine.g, q);
      bool nz = false;
#pragma unroll
      for (int k = 0; k < ZS; ++k) {
        bql[q * 64 * PER + k] = fmaf(delta_tx(r, dx[k], dy[k], dz[k], dp2[k]), fscf, gq);
        if constexpr (WTX) {
          const float wt = (q < qn && ink[k]) ? g.w_tx[(size_t)(q0 + q) * N + nk[k]] : 0.f;
          bql[q * 64 * PER + ZS + k] = wt;
          nz |= wt != 0.f;
        }
      }
      if (WTX && __ballot(nz) == 0ull) qact &= ~(1u << q);
    }
    for (int m0 = 0; m0 < M; m0 += 64) {
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
        float rm = 0.f;  // IQ: the receiver's phase term frac(fc/fs krx)
        if constexpr (IQ) {
          const double rv = g.fcfs * (double)krx;
          rm = (float)(rv - floor(rv));
        }
        float w[ZS], a[ZS];
        bool anyw = false;
#pragma unroll
        for (int k = 0; k < ZS; ++k) {
          w[k] = j < 0 ? 0.f : rx_weight(g, m, ex + dx[k], ey + dy[k], ez + dz[k]);
          a[k] = fmaf(delta_dist(ex, ey, ez, en, dx[k], dy[k], dz[k], dp2[k]), fscf, h);
          anyw |= w[k] != 0.f;
        }
        if (__ballot(anyw) == 0ull) continue;
        const S* cq = wtile + (size_t)q0 * q_el + (size_t)m * chan_el;
#pragma unroll 1
        for (int q = 0; q < QN; ++q) {
          if (!((qact >> q) & 1u)) continue;  // wavefront-uniform
          const bool live = q < qn;
          int t[ZS];
          uint32_t P[ZS], Plo[ZS];
          uint32_t Ps[IQ ? ZS : 1];
          int lo = BIG, hi = -BIG;
          float bqv[ZS], wqv[ZS];
#pragma unroll
          for (int k = 0; k < ZS; ++k) {
            bqv[k] = bql[q * 64 * PER + k];
            wqv[k] = WTX ? bql[q * 64 * PER + ZS + k] : 1.f;
          }
          const int ktxq = __builtin_amdgcn_readlane(my_ktx, q);
          const float rqq = IQ ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_rq), q)) : 0.f;
#pragma unroll
          for (int k = 0; k < ZS; ++k) {
            const float f = a[k] + bqv[k];
            t[k] = ktxq + krx + floor_i32(f);
            const float al = frac_f32(f);
            const bool valid = live && w[k] != 0.f && t[k] >= -1 && t[k] <= K - 1;
            const float wt = valid ? (WTX ? w[k] * wqv[k] : w[k]) : 0.f;
            if constexpr (IQ) {
              // revolutions fc/fs (ktx + krx + f) + fc t0, reduced to [0, 1)
              // before the hardware sine and cosine (which take revolutions)
              const float rev = frac_f32(rqq + rm + fcfs_f * f);
              const float wc = wt * __builtin_amdgcn_cosf(rev), wsn = wt * __builtin_amdgcn_sinf(rev);
              uint32_t unused;
              Mma<T>::pack2(wc - wc * al, wc * al, P[k], Plo[k]);
              Mma<T>::pack2(wsn - wsn * al, wsn * al, Ps[IQ ? k : 0], unused);
            } else {
              const float w2 = wt * al, w1 = wt - w2;
              Mma<T>::pack2(w1, w2, P[k], Plo[k]);
            }
            lo = valid ? min(lo, t[k]) : lo;
            hi = valid ? max(hi, t[k]) : hi;
            t[k] = valid ? t[k] : -BIG;
          }
          const int tmin = row_min(lo), tmax = row_max(hi);
          const bool any = tmax >= tmin;
          const int c_lo = any ? (tmin + CH) >> 3 : 0;  // chunk holding sample tmin
          const int nrow = any ? ((tmax + 1 + CH) >> 3) - c_lo + 1 : 0;
          const int nc = max(max(__builtin_amdgcn_readlane(nrow, 0), __builtin_amdgcn_readlane(nrow, 16)),
                             max(__builtin_amdgcn_readlane(nrow, 32), __builtin_amdgcn_readlane(nrow, 48)));
          const S* cqq = cq + (size_t)(live ? q : 0) * q_el;
          // slot of each tap relative to this row's chunk c_lo
          int d[ZS];
#pragma unroll
          for (int k = 0; k < ZS; ++k) d[k] = t[k] > -BIG ? t[k] + CH - CH * c_lo : -BIG;
          for (int u0 = 0; u0 < nc; u0 += NCH) {
            typename OP::Raw Br[NCH][NB];
            typename OP::Frag Bf[NCH][NB];
#pragma unroll
            for (int u = 0; u < NCH; ++u)
              if (u0 + u < nc) {
                const S* pc = cqq + (size_t)min(c_lo + u0 + u, Kc - 1) * chunk_el;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) Br[u][nb] = OP::load(pc + nb * 16 * CH);
              }
#pragma unroll
            for (int u = 0; u < NCH; ++u)
              if (u0 + u < nc) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) Bf[u][nb] = OP::decode(Br[u][nb]);
              }
#pragma unroll
            for (int k = 0; k < ZS; ++k) {
#pragma unroll
              for (int u = 0; u < NCH; ++u) {
                if (u0 + u >= nc) continue;
                const int du = d[k] - CH * (u0 + u);
                // does any lane hold a tap of group k in this chunk?
                if (__ballot((unsigned)(du + 1) <= (unsigned)CH) == 0ull) continue;
                const typename Mma<T>::Frag A = Mma<T>::place(P[k], du);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[k][nb] = Mma<T>::mma(A, Bf[u][nb], acc[k][nb]);
                if constexpr (IQ) {
                  const typename Mma<T>::Frag As = Mma<T>::place(Ps[IQ ? k : 0], du);
#pragma unroll
                  for (int nb = 0; nb < NB; ++nb)
                    acs[IQ ? k : 0][IQ ? nb : 0] = Mma<T>::mma(As, Bf[u][nb], acs[IQ ? k : 0][IQ ? nb : 0]);
                }
                if constexpr (Mma<T>::kSplit) {
                  const typename Mma<T>::Frag Al = Mma<T>::place(Plo[k], du);
#pragma unroll
                  for (int nb = 0; nb < NB; ++nb) acc[k][nb] = Mma<T>::mma(Al, Bf[u][nb], acc[k][nb]);
                }
              }
            }
          }
        }
      }
    }
  }
  // lane (vi, row) holds rows 4 row .. 4 row + 3 of column vi of each tile:
  // voxels (r, row) of each group, batch item vi of each tile
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int b = tile * TW + col0 + nb * 16 + vi;
    int e = 0;  // FP8: the item was stored as y 2^e
    if constexpr (__is_same(S, uint8_t)) e = fp8_item_exponent(g.amax[min(b, B - 1)]);
    if constexpr (IQ) {
      // each lane removes its own item's scale, then I = cos(I) - sin(Q) on
      // even columns and Q = sin(I) + cos(Q) on odd ones
#pragma unroll
      for (int k = 0; k < ZS; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float c = acc[k][nb][r], sn = acs[IQ ? k : 0][IQ ? nb : 0][r];
          if constexpr (__is_same(S, uint8_t)) {
            c = ldexpf(c * (1.f / Mma<T>::kScale), -e);
            sn = ldexpf(sn * (1.f / Mma<T>::kScale), -e);
          }
          const float ps = __shfl_xor(sn, 1);
          acc[k][nb][r] = (vi & 1) ? ps + c : c - ps;
        }
      e = 0;
    }
    if (b >= B) continue;
#pragma unroll
    for (int k = 0; k < ZS; ++k) {
      const int kx = k % GX, ky = (k / GX) % GY, kz = k / (GX * GY);
      const int jy = by0 + 4 * ky + row;
      if (gz0 + kz < 0 || jy >= g.n[1]) continue;
      float* xb = x + (size_t)b * N + (size_t)g.n[0] * (jy + (size_t)g.n[1] * (gz0 + kz));
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jx = bx0 + 4 * kx + r;
        if (jx < g.n[0]) {
          if constexpr (__is_same(S, uint8_t) && !IQ)
            xb[jx] = ldexpf(acc[k][nb][r] * (1.f / Mma<T>::kScale), -e);
          else
            xb[jx] = acc[k][nb][r];
        }
      }
    }
  }
}

// XCD-aware order: the hardware deals workgroups round-robin to the 8 XCDs of
// the chip, each with its own L2.  Remap so that every XCD receives runs of 128
// consecutive blocks (512 neighbouring wavefront columns, which read
// overlapping sample chunks); runs stay interleaved across XCDs, which keeps
// the depth-dependent work balanced.  The ragged last round keeps its order.
__device__ inline int xcd_remap(int b, int nblocks) {
  constexpr int X = 8, C = 128, per = X * C;
  if (b >= nblocks / per * per) return b;
  const int r = b / per, k = b - r * per;
  return r * per + (k % X) * C + k / X;
}

// Complex baseband doubles the accumulators: its bodies get the register
// budget of two wavefronts per SIMD (at three, some spilled).
template <class T, class BX, int NB, int QN, bool WTX, class OP, bool IQ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB == 4 || IQ ? 2 : 3))) void mfma_forward_stack(
    Geom g, const T* __restrict__ ws, int B, int TW, int Kc, float* __restrict__ x, int ngx,
    int ngy, int ncols) {
  __shared__ __align__(16) float bq_lds[4 * QN * 64 * BX::ZS * (WTX ? 2 : 1)];
  const int col = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (col >= ncols) return;  // whole wavefront
  stack_body<T, BX, NB, QN, WTX, OP, IQ>(g, ws, B, TW, Kc, x, ngx, ngy, col, blockIdx.y, bq_lds);
}

// Voxel groups per wavefront box: a 4 x 4 x 4 column (four 4 x 4 groups
// stacked in depth).
using kBox = Box<1, 1, 4>;
constexpr int kStack = kBox::ZS;

// Persistent form with dynamic scheduling.  Work items are (plan, wavefront
// column, 16-item batch slice), plan i owning items first[i] .. first[i+1]-1
// (columns fastest, deepest first).  The list is cut into runs of kRun
// consecutive items dealt round-robin to the 8 XCDs (run j to XCD j mod 8);
// each wavefront takes the next item of its XCD's runs from that XCD's
// counter (one atomic per item), so neighbouring columns share an L2 and the
// load balances dynamically, as hardware dispatch does for ordinary launches.
// Each item runs the same body as a single-plan launch, so results are
// identical bit for bit.  The counters are zeroed by zero_counters on the
// same stream before every launch.
constexpr unsigned kXcds = 8, kRun = 512;

__global__ void zero_counters(unsigned* c) {
  if (threadIdx.x < kXcds) c[threadIdx.x] = 0u;
}

template <class T, int QN, bool WTX, int NBMAX, bool IQ = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NBMAX == 4 || IQ ? 2 : 3))) void mfma_forward_batched(
    MfmaBatchedArgs a, unsigned* __restrict__ ctr) {
  __shared__ __align__(16) float bq_lds[4 * QN * 64 * kStack * (WTX ? 2 : 1)];
  const long long total = a.first[a.count];
  const unsigned xcd = blockIdx.x % kXcds;  // workgroups are dealt round-robin to the XCDs
  for (;;) {
    unsigned n = 0u;
    if ((threadIdx.x & 63) == 0) n = atomicAdd(ctr + xcd, 1u);
    n = __builtin_amdgcn_readfirstlane(n);
    const long long v = ((long long)(n / kRun) * kXcds + xcd) * kRun + n % kRun;
    if (v >= total) break;  // every later item of this XCD lies further on
    const int item = (int)v;
    int i = 0;
    while (item >= a.first[i + 1]) ++i;
    // copy the plan's share out of the argument block (uniform index: scalar
    // loads once per item, not a memory access per use in the loops)
    const MfmaWork w = a.p[i];
    const int local = item - a.first[i];
    const int col = local % w.ngroups, by = local / w.ngroups;
    // each plan runs with its own batch tiles per wavefront (w.nb, uniform:
    // NBMAX or 1)
    if (w.nb == NBMAX)
      stack_body<T, kBox, NBMAX, QN, WTX, Operand<T>, IQ>(w.g, static_cast<const T*>(w.ws), w.B,
                                                          w.TW, w.Kc, w.x, w.ngx, w.ngy, col, by,
                                                          bq_lds);
    else
      stack_body<T, kBox, 1, QN, WTX, Operand<T>, IQ>(w.g, static_cast<const T*>(w.ws), w.B, w.TW,
                                                      w.Kc, w.x, w.ngx, w.ngy, col, by, bq_lds);
  }
}

// y[nb][Q][M][K] f32 -> batch-tiled chunked workspace ws[Bp/TW][Q][M][Kc][TW][8]
// for items b0 .. b0+nb-1.  A workgroup converts 32 chunks (256 samples) of 16 items of
// one channel (q, m): rows of 256 samples are read coalesced into LDS (vec:
// K a multiple of 4 and y 16-byte aligned, each thread loads four samples of
// four rows with 16-byte loads, all issued before the LDS writes; else one
// sample of each row), then each thread packs two 8-sample chunks, the 16
// items of a chunk being adjacent 16-byte stores.
constexpr int RC = 32;  // chunks per reorder tile
template <class T>
__global__ __launch_bounds__(256) void reorder_chunks(const float* __restrict__ y, int Q, int M,
                                                      int K, int Kc, int nb, int b0, int TW,
                                                      T* __restrict__ ws,
                                                      const float* __restrict__ amax, int vec) {
  __shared__ float tile[16][RC * CH + 1];
  const long long QM = (long long)Q * M;
  const int t = threadIdx.x;
  const int kc0 = blockIdx.x * RC;
  const int i0 = blockIdx.z * 16;  // first item of this tile (relative to b0)
  for (long long qm = blockIdx.y; qm < QM; qm += gridDim.y) {
    if (vec) {
      // rows r, r + 4, r + 8, r + 12; samples 4 (t % 64) .. +3 of the tile.
      // With K a multiple of 4 the four samples are all inside [0, K) or all
      // outside (the tile starts at a multiple of 8).
      const int r = t >> 6, k4 = (t & 63) * 4;
      const int k = CH * (kc0 - 1) + k4;
      f32x4 v[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int b = i0 + r + 4 * p;
        v[p] = (b < nb && k >= 0 && k < K)
                   ? *reinterpret_cast<const f32x4*>(y + ((long long)b * QM + qm) * K + k)
                   : f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int c = 0; c < 4; ++c) tile[r + 4 * p][k4 + c] = v[p][c];
    } else {
      const int k = CH * (kc0 - 1) + t;
#pragma unroll 4
      for (int i = 0; i < 16; ++i) {
        const int b = i0 + i;
        tile[i][t] = (b < nb && k >= 0 && k < K) ? y[((long long)b * QM + qm) * K + k] : 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int o = t + 256 * j;
      const int kcl = o >> 4, i = o & 15;
      const int kc = kc0 + kcl, b = i0 + i;
      if (kc < Kc && b < nb) {
        const int ba = b0 + b, bt = ba / TW;
        T* dst = ws + (((long long)bt * QM + qm) * Kc + kc) * TW * CH + (long long)(ba - bt * TW) * CH;
        uint32_t v[CH];
        if constexpr (__is_same(T, uint8_t)) {
          // FP8: the item is stored as y 2^e
          const int e = fp8_item_exponent(amax[ba]);
#pragma unroll
          for (int s = 0; s < CH; ++s) v[s] = e4m3_bits(ldexpf(tile[i][kcl * CH + s], e));
          *reinterpret_cast<u32x2*>(dst) = u32x2{v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24),
                                                 v[4] | (v[5] << 8) | (v[6] << 16) | (v[7] << 24)};
        } else {
#pragma unroll
          for (int s = 0; s < CH; ++s) {
            const float f = tile[i][kcl * CH + s];
            if constexpr (__is_same(T, _Float16))
              v[s] = f16_bits(f);
            else
              v[s] = bf16_bits(f);
          }
          *reinterpret_cast<u32x4*>(dst) = u32x4{v[0] | (v[1] << 16), v[2] | (v[3] << 16),
                                                 v[4] | (v[5] << 16), v[6] | (v[7] << 16)};
        }
      }
    }
    __syncthreads();
  }
}

template <class T, class BX, int NB, int QN, bool WTX, class OP, bool IQ>
hipError_t launch_stack_t(const Geom& g, const void* ws, int B, float* x, hipStream_t st) {
  const int ngx = (g.n[0] + 4 * BX::GX - 1) / (4 * BX::GX), ngy = (g.n[1] + 4 * BX::GY - 1) / (4 * BX::GY);
  const int ncols = ngx * ngy * ((g.n[2] + BX::GZ - 1) / BX::GZ);
  const int TW = mfma_tile_width(B), Kc = mfma_chunks(g.K);
  dim3 grid((ncols + 3) / 4, mfma_batch_pad(B) / (16 * NB));
  hipLaunchKernelGGL((mfma_forward_stack<T, BX, NB, QN, WTX, OP, IQ>), grid, dim3(256), 0, st, g,
                     static_cast<const T*>(ws), B, TW, Kc, x, ngx, ngy, ncols);
  return hipGetLastError();
}

template <class T, class BX, int NB, class OP, bool IQ = false>
hipError_t launch_stack(const Geom& g, const void* ws, int B, float* x, hipStream_t st) {
  constexpr int QMAX = BX::ZS >= 8 ? 4 : 8;
  const bool wtx = g.w_tx != nullptr;
  const int qg = g.Q == 1 ? 1 : (g.Q <= 4 || QMAX == 4) ? 4 : 8;
  if (qg == 1)
    return wtx ? launch_stack_t<T, BX, NB, 1, true, OP, IQ>(g, ws, B, x, st)
               : launch_stack_t<T, BX, NB, 1, false, OP, IQ>(g, ws, B, x, st);
  if (qg == 4)
    return wtx ? launch_stack_t<T, BX, NB, 4, true, OP, IQ>(g, ws, B, x, st)
               : launch_stack_t<T, BX, NB, 4, false, OP, IQ>(g, ws, B, x, st);
  return wtx ? launch_stack_t<T, BX, NB, QMAX, true, OP, IQ>(g, ws, B, x, st)
             : launch_stack_t<T, BX, NB, QMAX, false, OP, IQ>(g, ws, B, x, st);
}

template <class T, class BX, class OP = Operand<T>>
hipError_t launch_any(const Geom& g, const void* ws, int B, float* x, hipStream_t st) {
  if (mfma_stack_tiles(B) == 4) return launch_stack<T, BX, 4, OP>(g, ws, B, x, st);
  if (mfma_stack_tiles(B) == 2) return launch_stack<T, BX, 2, OP>(g, ws, B, x, st);
  return launch_stack<T, BX, 1, OP>(g, ws, B, x, st);
}

// Complex baseband: twice the accumulators, so at most two batch tiles per
// wavefront (a workspace tile of four is covered in two halves).
template <class T, class BX>
hipError_t launch_any_iq(const Geom& g, const void* ws, int B, float* x, hipStream_t st) {
  if (mfma_stack_tiles(B) >= 2) return launch_stack<T, BX, 2, Operand<T>, true>(g, ws, B, x, st);
  return launch_stack<T, BX, 1, Operand<T>, true>(g, ws, B, x, st);
}

// Wavefront boxes of the plain (non-persistent) launch: a 4 x 4 x 4 column or
// an 8 x 8 x 1 slab (four lateral groups at one depth, whose taps cluster
// more tightly: fewer chunk loads per voxel).
using kSlab = Box<2, 2, 1>;
template <class T, class OP = Operand<T>>
hipError_t launch_box(const Geom& g, const void* ws, int B, float* x, bool slab, hipStream_t st) {
  return slab ? launch_any<T, kSlab, OP>(g, ws, B, x, st) : launch_any<T, kBox, OP>(g, ws, B, x, st);
}

template <class T, int QN, bool WTX, int NBMAX, bool IQ>
hipError_t batched_t(const MfmaBatchedArgs& a, unsigned* ctr, int cus, hipStream_t st) {
  auto kern = mfma_forward_batched<T, QN, WTX, NBMAX, IQ>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
  if (e != hipSuccess) return e;
  // resident workgroups only (a multiple of 8, so that each XCD holds the same
  // number), never more wavefronts than items
  const int total = a.first[a.count];
  int grid = std::max(1, per_cu) * cus;
  grid = std::min(grid, std::max(8, (total + 3) / 4));
  grid = std::max(8, grid / 8 * 8);
  hipLaunchKernelGGL(zero_counters, dim3(1), dim3(64), 0, st, ctr);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, a, ctr);
  return hipGetLastError();
}

template <class T, int NBMAX, bool IQ = false>
hipError_t batched_any(const MfmaBatchedArgs& a, unsigned* ctr, int qn, bool wtx, int cus,
                       hipStream_t st) {
  constexpr int QMAX = kStack >= 8 ? 4 : 8;
  if (qn == 1)
    return wtx ? batched_t<T, 1, true, NBMAX, IQ>(a, ctr, cus, st)
               : batched_t<T, 1, false, NBMAX, IQ>(a, ctr, cus, st);
  if (qn <= 4)
    return wtx ? batched_t<T, 4, true, NBMAX, IQ>(a, ctr, cus, st)
               : batched_t<T, 4, false, NBMAX, IQ>(a, ctr, cus, st);
  return wtx ? batched_t<T, QMAX, true, NBMAX, IQ>(a, ctr, cus, st)
             : batched_t<T, QMAX, false, NBMAX, IQ>(a, ctr, cus, st);
}

// Largest batch tiles per wavefront in a persistent launch.  FP8 fragments are
// half the registers of 16-bit ones, so the four-tile body fits without spills
// next to the one-tile body; the 16-bit types keep the two-tile body (and
// three wavefronts per SIMD), which measured faster for them in this kernel.
// Complex baseband doubles the accumulators: two tiles for every type.
int batched_nbmax(int storage, bool iq) { return storage == DAS_STORE_FP8_E4M3 && !iq ? 4 : 2; }

// Batch tiles per wavefront of a plan in a persistent launch: the kernel's
// NBMAX body or the one-tile body.
int persistent_nb(int storage, int B, bool iq) {
  const int nbmax = batched_nbmax(storage, iq), tiles = mfma_stack_tiles(B);
  return tiles >= nbmax ? nbmax : nbmax == 2 ? tiles : 1;
}

}  // namespace

int mfma_tiles_per_wave(int B) { return B > 32 ? 4 : B > 16 ? 2 : 1; }
int mfma_stack_tiles(int B) { return mfma_tiles_per_wave(B); }
int mfma_tile_width(int B) { return 16 * mfma_tiles_per_wave(B); }
int mfma_batch_pad(int B) {
  const int tw = mfma_tile_width(B);
  return (B + tw - 1) / tw * tw;
}

size_t mfma_batched_counter_bytes() { return kXcds * sizeof(unsigned); }

// A single plan runs faster through the persistent kernel (dynamic balance of
// the depth-dependent work) when that kernel gives it the same batch tiles per
// wavefront as the stack launch at the same occupancy: always for the 16-bit
// types up to two tiles; for FP8 only with four tiles (its one-tile body in
// the four-tile kernel runs at two wavefronts per SIMD instead of three).
bool mfma_prefers_persistent(int storage, int B) {
  const int nbmax = batched_nbmax(storage, false), tiles = mfma_stack_tiles(B);
  return nbmax == 2 ? tiles <= 2 : tiles == nbmax;
}

hipError_t launch_mfma_batched(MfmaBatchedArgs& a, unsigned* ctr, int storage, bool iq, int cus,
                               hipStream_t st) {
  int qn = 1;
  bool wtx = false;
  a.first[0] = 0;
  for (int i = 0; i < a.count; ++i) {
    MfmaWork& w = a.p[i];
    const int Q = w.g.Q;
    qn = std::max(qn, Q == 1 ? 1 : Q <= 4 ? 4 : 16);
    wtx |= w.g.w_tx != nullptr;
    w.ngx = (w.g.n[0] + 4 * kBox::GX - 1) / (4 * kBox::GX);
    w.ngy = (w.g.n[1] + 4 * kBox::GY - 1) / (4 * kBox::GY);
    w.ngroups = w.ngx * w.ngy * ((w.g.n[2] + kBox::GZ - 1) / kBox::GZ);  // wavefront boxes
    w.nbx = 0;
    w.nb = persistent_nb(storage, w.B, iq);
    a.first[i + 1] = a.first[i] + w.ngroups * (mfma_batch_pad(w.B) / (16 * w.nb));
  }
  // complex baseband (every plan of the launch; f16 or FP8 storage)
  if (iq && storage == DAS_STORE_F16) return batched_any<_Float16, 2, true>(a, ctr, qn, wtx, cus, st);
  if (iq) return batched_any<uint8_t, 2, true>(a, ctr, qn, wtx, cus, st);
  if (storage == DAS_STORE_F16) return batched_any<_Float16, 2>(a, ctr, qn, wtx, cus, st);
  if (storage == DAS_STORE_FP8_E4M3) return batched_any<uint8_t, 4>(a, ctr, qn, wtx, cus, st);
  return batched_any<uint16_t, 2>(a, ctr, qn, wtx, cus, st);
}
int mfma_chunks(int K) { return (K + CH - 1) / CH + 2; }

size_t mfma_workspace_elems(const Geom& g, int B) {
  return (size_t)g.Q * g.M * mfma_chunks(g.K) * mfma_batch_pad(B) * CH;
}

hipError_t launch_mfma_reorder(const Geom& g, int storage, const float* y, int b0, int nb, int btot,
                               void* ws, hipStream_t st) {
  const int Kc = mfma_chunks(g.K), TW = mfma_tile_width(btot);
  const long long QM = (long long)g.Q * g.M;
  // at most 1024 channel rows of blocks, each block looping over channels
  // (cfg2, 256 frames f16: 13.7 -> 12.0-12.9 ms against one block per channel)
  const dim3 grid((Kc + RC - 1) / RC, (unsigned)std::min<long long>(QM, 1024), (nb + 15) / 16);
  const int vec = g.K % 4 == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0;
  if (storage == DAS_STORE_F16) {
    hipLaunchKernelGGL(reorder_chunks<_Float16>, grid, dim3(256), 0, st, y, g.Q, g.M, g.K, Kc, nb,
                       b0, TW, static_cast<_Float16*>(ws), nullptr, vec);
  } else if (storage == DAS_STORE_FP8_E4M3) {
    hipError_t e = launch_item_absmax(g, y, b0, nb, const_cast<float*>(g.amax), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reorder_chunks<uint8_t>, grid, dim3(256), 0, st, y, g.Q, g.M, g.K, Kc, nb,
                       b0, TW, static_cast<uint8_t*>(ws), g.amax, vec);
  } else {
    hipLaunchKernelGGL(reorder_chunks<uint16_t>, grid, dim3(256), 0, st, y, g.Q, g.M, g.K, Kc, nb,
                       b0, TW, static_cast<uint16_t*>(ws), nullptr, vec);
  }
  return hipGetLastError();
}

hipError_t launch_mfma_forward_iq(const Geom& g, int storage, const void* ws, int B, float* x,
                                  bool slab, hipStream_t st) {
  if (storage == DAS_STORE_F16)
    return slab ? launch_any_iq<_Float16, kSlab>(g, ws, B, x, st) : launch_any_iq<_Float16, kBox>(g, ws, B, x, st);
  if (storage == DAS_STORE_FP8_E4M3)
    return slab ? launch_any_iq<uint8_t, kSlab>(g, ws, B, x, st) : launch_any_iq<uint8_t, kBox>(g, ws, B, x, st);
  return hipErrorInvalidValue;  // bf16: not built (split weights)
}

hipError_t launch_mfma_forward(const Geom& g, int storage, const void* ws, int B, float* x,
                               bool slab, bool fp8_operands, hipStream_t st) {
  if (storage == DAS_STORE_F16) return launch_box<_Float16>(g, ws, B, x, slab, st);
  if (storage == DAS_STORE_FP8_E4M3)
    return fp8_operands ? launch_box<uint8_t, OperandFp8Raw>(g, ws, B, x, slab, st)
                        : launch_box<uint8_t>(g, ws, B, x, slab, st);
  return launch_box<uint16_t>(g, ws, B, x, slab, st);
}

}  // namespace dasmi
