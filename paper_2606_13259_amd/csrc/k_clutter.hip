// Rank-truncation (SVD) clutter filter and power Doppler of a beamformed
// ensemble: the rank-truncation primitive that the paper names beside its
// beamformer (Sec. 1, Sec. 5).  The ensemble x[T][N] (T frames of N voxels)
// is the Casorati matrix S = x^T (N x T); S = U diag(sigma) V^T; the filter
// keeps the singular components k_lo .. k_hi-1 and the power Doppler image is
// P[n] = (1/T) sum_t xf[t][n]^2.
//
// MI355X design (T <= 512 frames, N voxels):
//   1. Gram matrix G = x x^T (T x T), the only O(N T^2) step: a dense
//      contraction over voxels on the matrix cores (v_mfma_f32_16x16x4_f32,
//      FP32 products and partial sums over one voxel chunk), chunks merged in
//      FP64 with atomics.  Workgroups own a 64 x 64 block of G (upper
//      triangle only) for one voxel chunk; the two 64-frame row panels of a
//      64-voxel step are staged through LDS with coalesced loads.
//   2. Eigen-decomposition G = V diag(lambda) V^T by the parallel cyclic
//      Jacobi method (round-robin pairing, T/2 disjoint rotations per round)
//      in one workgroup.  T <= 256: the matrix lives in that CU's LDS (upper
//      triangle, FP32), the rotations are logged and replayed on the rows of
//      V afterwards (FP64); T > 256: matrix and V in global memory (FP64,
//      much slower: every round waits on L2).  sigma = sqrt(lambda), sorted;
//      the columns of V that the filter needs are copied (FP32) as the
//      projection basis B.
//   3. Projection and power: per voxel, a = B^T s_n, then the filtered
//      series is B a (keep form) or s_n - B a (removal form), whichever uses
//      fewer components (at most 64), and P[n] its mean square.  Every voxel
//      reads its T samples twice (from L2 or HBM); B sits in LDS.
#include <mutex>

#include "das_internal.h"

namespace dasmi {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int GB = 64;  // Gram block (frames) per workgroup, and voxels per step

__global__ void zero_f64(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// G[i][j] += sum over this workgroup's voxel chunk of x[i][n] x[j][n], for
// the frame blocks (I, J), I <= J (blockIdx.x enumerates the pairs), voxel
// chunk blockIdx.y of `csz` voxels.  Wavefront w computes the 32 x 32
// sub-block (rows 32 (w / 2), columns 32 (w % 2)) as 2 x 2 MFMA tiles.
__global__ __launch_bounds__(256) void gram_mfma(const float* __restrict__ x, int T, long long N,
                                                 long long csz, int nbk, double* __restrict__ G) {
  __shared__ float XI[GB][GB + 1], XJ[GB][GB + 1];
  // pair index -> (I, J), I <= J
  int I = 0, rem = blockIdx.x;
  while (rem >= nbk - I) {
    rem -= nbk - I;
    ++I;
  }
  const int J = I + rem;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int rb = 32 * (wave >> 1), cb = 32 * (wave & 1);
  const long long v0 = (long long)blockIdx.y * csz;
  const long long v1 = min(N, v0 + csz);
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (long long s = v0; s < v1; s += GB) {
    __syncthreads();  // the previous step's panels are no longer read
#pragma unroll
    for (int i = 0; i < GB * GB / 256; ++i) {
      const int idx = t + 256 * i;
      const int r = idx / GB, c = idx % GB;
      const long long v = s + c;
      const int fi = I * GB + r, fj = J * GB + r;
      XI[r][c] = (v < v1 && fi < T) ? x[(long long)fi * N + v] : 0.f;
      XJ[r][c] = (v < v1 && fj < T) ? x[(long long)fj * N + v] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GB / 4; ++kk) {
      const int k = 4 * kk + (lane >> 4);
      float a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        a[u] = XI[rb + 16 * u + (lane & 15)][k];
        b[u] = XJ[cb + 16 * u + (lane & 15)][k];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
          acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[v], acc[u][v], 0, 0, 0);
    }
  }
  // D[i][j] of a tile: lane holds rows 4 (lane / 16) + r, column lane % 16
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * GB + rb + 16 * u + 4 * (lane >> 4) + r;
        const int j = J * GB + cb + 16 * v + (lane & 15);
        if (i < T && j < T && i <= j) atomicAdd(G + (size_t)i * T + j, (double)acc[u][v][r]);
      }
}

// A(i, j) of the symmetric matrix kept in the upper triangle of a.
__device__ inline double& up(double* a, int T, int i, int j) {
  return i <= j ? a[(size_t)i * T + j] : a[(size_t)j * T + i];
}

// Parallel cyclic Jacobi on the T x T symmetric matrix a (upper triangle,
// overwritten: its diagonal ends as the eigenvalues) with eigenvectors
// accumulated in v (T x T, columns).  One workgroup of 1024 threads.
// Round r pairs the indices by the round-robin (circle) schedule over
// Tp = T rounded up to even (index T, if present, is a dummy that never
// rotates).  Per round: the T/2 rotations are formed (each pair also updates
// its own 2 x 2 diagonal block in closed form), then every off-diagonal 2 x 2
// block between two pairs becomes R1^T M R2 and the columns p, q of v rotate.
// Sweeps stop when the off-diagonal mass falls below 1e-26 of the diagonal
// mass (squares), or after 40 sweeps.  Then the eigenvalues are ranked
// (descending, ties by index), sigma = sqrt(max(lambda, 0)) is written, and
// the basis columns (ranks [k_lo, k_hi) for keep, the others for removal) are
// copied to B[T][nb] in FP32.
__global__ __launch_bounds__(1024) void jacobi_eig(double* __restrict__ a, double* __restrict__ v,
                                                   int T, int k_lo, int k_hi, int keep,
                                                   float* __restrict__ sv, float* __restrict__ Bm,
                                                   int nb) {
  constexpr int MAXP = 256;  // pairs (T <= 512)
  __shared__ int P[MAXP], Q[MAXP];
  __shared__ double C[MAXP], S[MAXP];
  __shared__ double red[2][32];
  __shared__ int rank_of[512];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int Tp = T + (T & 1), np = Tp / 2;
  for (int i = tid; i < T * T; i += nt) v[i] = (i / T == i % T) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    for (int r = 0; r < Tp - 1; ++r) {
      if (tid < np) {
        auto pos = [&](int k) { return k == 0 ? 0 : 1 + (k - 1 + r) % (Tp - 1); };
        int p = pos(tid), q = pos(Tp - 1 - tid);
        if (p > q) {
          const int w = p;
          p = q;
          q = w;
        }
        double c = 1.0, s = 0.0;
        if (q < T) {
          const double app = up(a, T, p, p), aqq = up(a, T, q, q), apq = up(a, T, p, q);
          if (apq != 0.0) {
            const double th = (aqq - app) / (2.0 * apq);
            const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            s = tt * c;
            up(a, T, p, p) = app - tt * apq;
            up(a, T, q, q) = aqq + tt * apq;
            up(a, T, p, q) = 0.0;
          }
        }
        P[tid] = p;
        Q[tid] = q;
        C[tid] = c;
        S[tid] = s;
      }
      __syncthreads();
      // off-diagonal blocks between pairs k1 < k2
      const int nblk = np * (np - 1) / 2;
      for (int w = tid; w < nblk; w += nt) {
        int k2 = (int)((1.0 + sqrt(1.0 + 8.0 * (double)w)) * 0.5);
        while (k2 * (k2 - 1) / 2 > w) --k2;
        while ((k2 + 1) * k2 / 2 <= w) ++k2;
        const int k1 = w - k2 * (k2 - 1) / 2;
        const int p1 = P[k1], q1 = Q[k1], p2 = P[k2], q2 = Q[k2];
        const double c1 = C[k1], s1 = S[k1], c2 = C[k2], s2 = S[k2];
        if ((s1 == 0.0 && s2 == 0.0) || p1 >= T || p2 >= T) continue;
        const bool q1v = q1 < T, q2v = q2 < T;
        const double m00 = up(a, T, p1, p2);
        const double m01 = q2v ? up(a, T, p1, q2) : 0.0;
        const double m10 = q1v ? up(a, T, q1, p2) : 0.0;
        const double m11 = (q1v && q2v) ? up(a, T, q1, q2) : 0.0;
        // rows (p1, q1) by R1, then columns (p2, q2) by R2
        const double b00 = c1 * m00 - s1 * m10, b01 = c1 * m01 - s1 * m11;
        const double b10 = s1 * m00 + c1 * m10, b11 = s1 * m01 + c1 * m11;
        up(a, T, p1, p2) = c2 * b00 - s2 * b01;
        if (q2v) up(a, T, p1, q2) = s2 * b00 + c2 * b01;
        if (q1v) up(a, T, q1, p2) = c2 * b10 - s2 * b11;
        if (q1v && q2v) up(a, T, q1, q2) = s2 * b10 + c2 * b11;
      }
      // eigenvector columns
      for (int w = tid; w < np * T; w += nt) {
        const int k = w / T, i = w - k * T;
        const int p = P[k], q = Q[k];
        const double c = C[k], s = S[k];
        if (s == 0.0 || q >= T) continue;
        const double vp = v[(size_t)i * T + p], vq = v[(size_t)i * T + q];
        v[(size_t)i * T + p] = c * vp - s * vq;
        v[(size_t)i * T + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    // convergence: off-diagonal vs diagonal mass
    double off = 0.0, dia = 0.0;
    for (int w = tid; w < T * T; w += nt) {
      const int i = w / T, j = w - i * T;
      const double e = a[w];
      if (i < j) off += e * e;
      if (i == j) dia += e * e;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      dia += __shfl_xor(dia, o);
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = off;
      red[1][tid >> 6] = dia;
    }
    __syncthreads();
    off = 0.0;
    dia = 0.0;
    for (int w = 0; w < nt / 64; ++w) {
      off += red[0][w];
      dia += red[1][w];
    }
    __syncthreads();
    if (off <= 1e-26 * dia) break;  // uniform: every thread read the same sums
  }
  // rank the eigenvalues, descending (ties by index)
  for (int i = tid; i < T; i += nt) {
    const double li = a[(size_t)i * T + i];
    int rk = 0;
    for (int j = 0; j < T; ++j) {
      const double lj = a[(size_t)j * T + j];
      rk += (lj > li) || (lj == li && j < i);
    }
    rank_of[rk] = i;
    sv[rk] = (float)sqrt(fmax(li, 0.0));
  }
  __syncthreads();
  // basis columns: ranks in [k_lo, k_hi) (keep) or outside it (removal)
  for (int w = tid; w < T * nb; w += nt) {
    const int t = w / nb, j = w - t * nb;
    const int rk = keep ? k_lo + j : (j < k_lo ? j : k_hi + (j - k_lo));
    Bm[w] = (float)v[(size_t)t * T + rank_of[rk]];
  }
}

// ---------------------------------------------------------------------------
// Fast path for T <= 256: the same parallel Jacobi with the matrix in LDS.
// The upper triangle in FP32 (T (T+1)/2 floats, at most 128.5 KiB) stays in
// one CU's LDS for all sweeps; every rotation (c, s, p, q) is logged to
// global memory and the eigenvectors are formed afterwards by replaying the
// log on the rows of V (rows evolve independently: row i only ever mixes its
// own entries p and q), in FP64, one row per thread.  FP32 is ample here:
// the eigenvalues are needed to a small fraction of sigma_1^2 and the
// eigenvectors only across the gaps at the cuts.
constexpr int kFastT = 256;
constexpr int kMaxSweeps = 30;

struct Rot {
  float c, s;
  short p, q;
};

__device__ inline int upk(int T, int i, int j) {  // packed upper-triangle index, i <= j
  return i * T - (i * (i - 1)) / 2 + (j - i);
}
__device__ inline float& upl(float* a, int T, int i, int j) {
  return i <= j ? a[upk(T, i, j)] : a[upk(T, j, i)];
}

__global__ __launch_bounds__(1024) void jacobi_lds(const double* __restrict__ G, int T,
                                                   Rot* __restrict__ log, int* __restrict__ nrot,
                                                   float* __restrict__ lam) {
  extern __shared__ float A[];  // T (T+1)/2
  __shared__ int P[kFastT / 2], Q[kFastT / 2];
  __shared__ float C[kFastT / 2], S[kFastT / 2];
  __shared__ float red[2][16];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int Tp = T + (T & 1), np = Tp / 2;
  for (int w = tid; w < T * T; w += nt) {
    const int i = w / T, j = w - i * T;
    if (i <= j) A[upk(T, i, j)] = (float)G[w];
  }
  __syncthreads();
  __shared__ int rotated;
  if (tid == 0) rotated = 0;
  __syncthreads();
  int sweeps = 0;
  for (; sweeps < kMaxSweeps; ++sweeps) {
    for (int r = 0; r < Tp - 1; ++r) {
      if (tid < np) {
        auto pos = [&](int k) { return k == 0 ? 0 : 1 + (k - 1 + r) % (Tp - 1); };
        int p = pos(tid), q = pos(Tp - 1 - tid);
        if (p > q) {
          const int w = p;
          p = q;
          q = w;
        }
        float c = 1.f, s = 0.f;
        if (q < T) {
          const float app = upl(A, T, p, p), aqq = upl(A, T, q, q), apq = upl(A, T, p, q);
          if (fabsf(apq) > 1.1920929e-7f * sqrtf(fabsf(app * aqq))) {
            rotated = 1;
            const float th = (aqq - app) / (2.f * apq);
            const float tt = (th >= 0.f ? 1.f : -1.f) / (fabsf(th) + sqrtf(th * th + 1.f));
            c = 1.f / sqrtf(tt * tt + 1.f);
            s = tt * c;
            upl(A, T, p, p) = app - tt * apq;
            upl(A, T, q, q) = aqq + tt * apq;
            upl(A, T, p, q) = 0.f;
          }
        }
        P[tid] = p;
        Q[tid] = q;
        C[tid] = c;
        S[tid] = s;
        log[((size_t)sweeps * (Tp - 1) + r) * np + tid] = Rot{c, s, (short)p, (short)q};
      }
      __syncthreads();
      const int nblk = np * (np - 1) / 2;
      for (int w = tid; w < nblk; w += nt) {
        int k2 = (int)((1.f + sqrtf(1.f + 8.f * (float)w)) * 0.5f);
        while (k2 * (k2 - 1) / 2 > w) --k2;
        while ((k2 + 1) * k2 / 2 <= w) ++k2;
        const int k1 = w - k2 * (k2 - 1) / 2;
        const float s1 = S[k1], s2 = S[k2];
        if (s1 == 0.f && s2 == 0.f) continue;
        const int p1 = P[k1], q1 = Q[k1], p2 = P[k2], q2 = Q[k2];
        const float c1 = C[k1], c2 = C[k2];
        const bool q1v = q1 < T, q2v = q2 < T;
        const float m00 = upl(A, T, p1, p2);
        const float m01 = q2v ? upl(A, T, p1, q2) : 0.f;
        const float m10 = q1v ? upl(A, T, q1, p2) : 0.f;
        const float m11 = (q1v && q2v) ? upl(A, T, q1, q2) : 0.f;
        const float b00 = c1 * m00 - s1 * m10, b01 = c1 * m01 - s1 * m11;
        const float b10 = s1 * m00 + c1 * m10, b11 = s1 * m01 + c1 * m11;
        upl(A, T, p1, p2) = c2 * b00 - s2 * b01;
        if (q2v) upl(A, T, p1, q2) = s2 * b00 + c2 * b01;
        if (q1v) upl(A, T, q1, p2) = c2 * b10 - s2 * b11;
        if (q1v && q2v) upl(A, T, q1, q2) = s2 * b10 + c2 * b11;
      }
      __syncthreads();
    }
    float off = 0.f, dia = 0.f;
    for (int w = tid; w < T * T; w += nt) {
      const int i = w / T, j = w - i * T;
      if (i < j) {
        const float e = A[upk(T, i, j)];
        off += e * e;
      } else if (i == j) {
        const float e = A[upk(T, i, i)];
        dia += e * e;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      dia += __shfl_xor(dia, o);
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = off;
      red[1][tid >> 6] = dia;
    }
    __syncthreads();
    off = 0.f;
    dia = 0.f;
    for (int w = 0; w < nt / 64; ++w) {
      off += red[0][w];
      dia += red[1][w];
    }
    __syncthreads();
    // converged: off-diagonal mass negligible, or a whole sweep without a
    // rotation (every |a_pq| <= 2^-23 sqrt(a_pp a_qq): the relative
    // criterion, which keeps refining the small eigenpairs)
    const bool none = rotated == 0;
    __syncthreads();
    if (off <= 1e-13f * dia || none) {
      ++sweeps;
      break;
    }
    if (tid == 0) rotated = 0;
    __syncthreads();
  }
  for (int i = tid; i < T; i += nt) lam[i] = A[upk(T, i, i)];
  if (tid == 0) *nrot = sweeps * (Tp - 1) * np;
}

// V = product of the logged rotations, row by row: row i starts as e_i and
// every rotation (c, s, p, q) mixes its entries p and q.  Rows are
// independent, and the rotations of one round touch disjoint entries, so one
// wavefront replays one row with its lanes sharing each round's rotations
// (lane l takes pairs l, l + 64, ...); the rounds run in program order on the
// row held in LDS (one wavefront: LDS operations stay in order, no barrier).
__global__ __launch_bounds__(64) void replay_rotations(const Rot* __restrict__ log,
                                                       const int* __restrict__ nrot, int T,
                                                       double* __restrict__ v) {
  __shared__ double row[kFastT];
  const int lane = threadIdx.x, i = blockIdx.x;
  const int np = (T + (T & 1)) / 2;
  for (int j = lane; j < T; j += 64) row[j] = (j == i) ? 1.0 : 0.0;
  __builtin_amdgcn_wave_barrier();
  const int nrounds = *nrot / np;
  for (int k = 0; k < nrounds; ++k) {
    const Rot* rk = log + (size_t)k * np;
    for (int j = lane; j < np; j += 64) {
      const Rot r = rk[j];
      if (r.s == 0.f || r.q >= T) continue;
      // renormalised in FP64: FP32 (c, s) have c^2 + s^2 = 1 +- 1e-7, and a
      // row meets thousands of rotations
      const double inv = 1.0 / sqrt((double)r.c * r.c + (double)r.s * r.s);
      const double c = r.c * inv, s = r.s * inv;
      const double vp = row[r.p], vq = row[r.q];
      row[r.p] = c * vp - s * vq;
      row[r.q] = s * vp + c * vq;
    }
    __builtin_amdgcn_wave_barrier();  // round k's updates precede round k + 1's reads
  }
  for (int j = lane; j < T; j += 64) v[(size_t)i * T + j] = row[j];
}

// Rank the eigenvalues lam (descending, ties by index), write sigma, and form
// the projection basis B[T][nb] (ranks [k_lo, k_hi) for keep, the others for
// removal), refined in FP64 across the cuts.  The FP32 Jacobi leaves each
// eigenvector accurate to about the FP32 rounding of the matrix; the filter
// only depends on the split between the basis set D and its complement K, so
// one first-order correction with the FP64 Gram matrix G removes that error:
//   W = G V_D,   delta_id = v_i . W_d,   b_d = v_d + sum_{i in K} v_i delta_id / (lam_d - lam_i)
// (second-order terms, (delta / gap)^2, are far below FP32).  Pairs closer
// than 1e-6 lam_max are not corrected (no gap: the split is not unique
// there).  G's storage is reused for the coefficients E once W is formed.
__global__ __launch_bounds__(1024) void rank_refine_basis(const float* __restrict__ lam,
                                                          const double* __restrict__ v, double* G,
                                                          double* __restrict__ W, int T, int k_lo,
                                                          int k_hi, int keep, float* __restrict__ sv,
                                                          float* __restrict__ Bm, int nb) {
  __shared__ int rank_of[kFastT], D[64], Kset[kFastT];
  __shared__ unsigned char inD[kFastT];
  __shared__ float lmax;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < T; i += nt) {
    const float li = lam[i];
    int rk = 0;
    for (int j = 0; j < T; ++j) {
      const float lj = lam[j];
      rk += (lj > li) || (lj == li && j < i);
    }
    rank_of[rk] = i;
    sv[rk] = sqrtf(fmaxf(li, 0.f));
    inD[i] = 0;
  }
  __syncthreads();
  if (tid == 0) lmax = fmaxf(lam[rank_of[0]], 0.f);
  for (int j = tid; j < nb; j += nt) {
    const int rk = keep ? k_lo + j : (j < k_lo ? j : k_hi + (j - k_lo));
    D[j] = rank_of[rk];
  }
  __syncthreads();
  for (int j = tid; j < nb; j += nt) inD[D[j]] = 1;
  __syncthreads();
  if (tid == 0) {
    int c = 0;
    for (int i = 0; i < T; ++i)
      if (!inD[i]) Kset[c++] = i;
  }
  __syncthreads();
  const int nK = T - nb;
  // W = G V_D
  for (int w = tid; w < T * nb; w += nt) {
    const int t = w / nb, j = w - t * nb;
    const int d = D[j];
    double acc = 0.0;
    for (int u = 0; u < T; ++u) acc += up(G, T, t, u) * v[(size_t)u * T + d];
    W[w] = acc;
  }
  __syncthreads();
  // E[i][j] (i over K) into G's storage
  double* E = G;
  for (int w = tid; w < nK * nb; w += nt) {
    const int ii = w / nb, j = w - ii * nb;
    const int i = Kset[ii], d = D[j];
    double dl = 0.0;
    for (int t = 0; t < T; ++t) dl += v[(size_t)t * T + i] * W[t * nb + j];
    const double gap = (double)lam[d] - (double)lam[i];
    E[w] = fabs(gap) > 1e-6 * (double)lmax ? dl / gap : 0.0;
  }
  __syncthreads();
  for (int w = tid; w < T * nb; w += nt) {
    const int t = w / nb, j = w - t * nb;
    double b = v[(size_t)t * T + D[j]];
    for (int ii = 0; ii < nK; ++ii) b += v[(size_t)t * T + Kset[ii]] * E[ii * nb + j];
    Bm[w] = (float)b;
  }
}

// Per voxel n: a = B^T s_n, filtered series (keep: B a; removal: s_n - B a),
// P[n] = mean square; xf (optional) receives the filtered series.  B[T][nb]
// in LDS.  NBMAX >= nb.
template <int NBMAX>
__global__ __launch_bounds__(256) void project_power(const float* __restrict__ x, int T,
                                                     long long N, const float* __restrict__ Bm,
                                                     int nb, int keep, float* __restrict__ pd,
                                                     float* __restrict__ xf) {
  extern __shared__ float Bs[];
  for (int i = threadIdx.x; i < T * nb; i += blockDim.x) Bs[i] = Bm[i];
  __syncthreads();
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float acoef[NBMAX];
#pragma unroll
  for (int j = 0; j < NBMAX; ++j) acoef[j] = 0.f;
  for (int t = 0; t < T; ++t) {
    const float s = x[(long long)t * N + n];
#pragma unroll
    for (int j = 0; j < NBMAX; ++j)
      if (j < nb) acoef[j] = fmaf(s, Bs[t * nb + j], acoef[j]);
  }
  double pw = 0.0;
  for (int t = 0; t < T; ++t) {
    const float s = x[(long long)t * N + n];
    float pr = 0.f;
#pragma unroll
    for (int j = 0; j < NBMAX; ++j)
      if (j < nb) pr = fmaf(acoef[j], Bs[t * nb + j], pr);
    const float f = keep ? pr : s - pr;
    pw += (double)f * (double)f;
    if (xf) xf[(long long)t * N + n] = f;
  }
  pd[n] = (float)(pw / T);
}

template <int NBMAX>
hipError_t launch_project(const float* x, int T, long long N, const float* Bm, int nb, int keep,
                          float* pd, float* xf, hipStream_t st) {
  const size_t lds = sizeof(float) * (size_t)T * nb;
  auto kern = project_power<NBMAX>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)((N + 255) / 256)), dim3(256), lds, st, x, T, N, Bm, nb,
                     keep, pd, xf);
  return hipGetLastError();
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr size_t rot_log_bytes(int T) {
  const int Tp = T + (T & 1);
  return align256(sizeof(Rot) * (size_t)kMaxSweeps * (Tp - 1) * (Tp / 2));
}

constexpr size_t workspace_bytes(int T) {
  size_t b = 2 * align256(sizeof(double) * (size_t)T * T) + align256(sizeof(float) * (size_t)T * 64);
  if (T <= kFastT)
    b += rot_log_bytes(T) + align256(sizeof(float) * (size_t)T) + 256 +
         align256(sizeof(double) * (size_t)T * 64);
  return b;
}

// Workspace of the allocation-free entry point: room for ensembles of up to
// kStaticT frames (12.4 MiB), one copy per device, held until the process
// ends.  In host code `scratch` names a host-side stand-in, not the device
// array: its device address comes from hipGetSymbolAddress, once per device.
constexpr int kStaticT = 256;
constexpr size_t kStaticBytes = workspace_bytes(kStaticT);
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

}  // namespace

size_t clutter_workspace_bytes(int T) { return workspace_bytes(T); }

int clutter_static_max_frames() { return kStaticT; }

// Device address of this device's copy of `scratch`, looked up on the first
// call made with each device current and kept.
hipError_t clutter_static_scratch(void** ptr, size_t* bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kStaticBytes;
  return hipSuccess;
}

int clutter_basis_size(int T, int k_lo, int k_hi) {
  const int kept = k_hi - k_lo;
  return std::min(kept, T - kept);
}

hipError_t launch_clutter_filter(const float* x, int T, long long N, int k_lo, int k_hi, float* sv,
                                 float* pd, float* xf, void* ws, int cus, hipStream_t st) {
  char* w = static_cast<char*>(ws);
  double* G = reinterpret_cast<double*>(w);
  double* V = reinterpret_cast<double*>(w + align256(sizeof(double) * (size_t)T * T));
  float* Bm = reinterpret_cast<float*>(w + 2 * align256(sizeof(double) * (size_t)T * T));
  const int kept = k_hi - k_lo;
  const int keep = kept <= T - kept ? 1 : 0;
  const int nb = keep ? kept : T - kept;
  hipLaunchKernelGGL(zero_f64, dim3(256), dim3(256), 0, st, G, (size_t)T * T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nbk = (T + GB - 1) / GB, npairs = nbk * (nbk + 1) / 2;
  const long long nsteps = (N + GB - 1) / GB;
  const long long nchunk = std::max(1LL, std::min(nsteps, (long long)(8 * cus) / npairs + 1));
  const long long csz = (nsteps + nchunk - 1) / nchunk * GB;
  const long long nch = (N + csz - 1) / csz;
  hipLaunchKernelGGL(gram_mfma, dim3((unsigned)npairs, (unsigned)nch), dim3(256), 0, st, x, T, N,
                     csz, nbk, G);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (T <= kFastT) {
    char* w2 = w + 2 * align256(sizeof(double) * (size_t)T * T) + align256(sizeof(float) * (size_t)T * 64);
    Rot* log = reinterpret_cast<Rot*>(w2);
    float* lam = reinterpret_cast<float*>(w2 + rot_log_bytes(T));
    int* nrot = reinterpret_cast<int*>(w2 + rot_log_bytes(T) + align256(sizeof(float) * (size_t)T));
    const size_t lds = sizeof(float) * (size_t)T * (T + 1) / 2;
    if (lds > 65536) {
      e = hipFuncSetAttribute((const void*)jacobi_lds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(jacobi_lds, dim3(1), dim3(1024), lds, st, G, T, log, nrot, lam);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(replay_rotations, dim3(T), dim3(64), 0, st, log, nrot, T, V);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double* W = reinterpret_cast<double*>(w2 + rot_log_bytes(T) + align256(sizeof(float) * (size_t)T) + 256);
    hipLaunchKernelGGL(rank_refine_basis, dim3(1), dim3(1024), 0, st, lam, V, G, W, T, k_lo, k_hi, keep,
                       sv, Bm, nb);
  } else {
    hipLaunchKernelGGL(jacobi_eig, dim3(1), dim3(1024), 0, st, G, V, T, k_lo, k_hi, keep, sv, Bm, nb);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (nb == 0) {  // keep nothing or remove nothing
    return launch_project<1>(x, T, N, Bm, 0, keep, pd, xf, st);
  }
  if (nb <= 8) return launch_project<8>(x, T, N, Bm, nb, keep, pd, xf, st);
  if (nb <= 16) return launch_project<16>(x, T, N, Bm, nb, keep, pd, xf, st);
  if (nb <= 32) return launch_project<32>(x, T, N, Bm, nb, keep, pd, xf, st);
  return launch_project<64>(x, T, N, Bm, nb, keep, pd, xf, st);
}

}  // namespace dasmi
