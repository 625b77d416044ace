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
//      FP64 with atomics.  T <= 256: a workgroup forms the whole upper
//      triangle for its voxel chunk from one LDS stage of all frames, so the
//      ensemble is read once; larger T: workgroups own 64 x 64 blocks.
//   2. Eigen-decomposition G = V diag(lambda) V^T in FP64: Householder
//      tridiagonalisation (one workgroup, matrix in L2), all eigenvalues by
//      multisection on Sturm counts (one wavefront each), and the
//      eigenvectors that the filter uses (at most 64) by inverse iteration
//      in LDS, re-orthogonalised within clusters and back-transformed by the
//      reflectors.  sigma = sqrt(lambda), sorted; those columns of V are
//      the projection basis B (FP32 and FP64).
//   3. Projection and power: per voxel, a = B^T s_n, then the filtered
//      series is B a (keep form) or s_n - B a (removal form), whichever uses
//      fewer components (at most 64), and P[n] its mean square.  When only
//      the power is asked for (and the basis is small), one FP64 pass gives
//      it from |a|^2 and |s_n|^2; otherwise every voxel reads its T samples
//      twice (from L2 or HBM).  B sits in LDS.
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

// T <= 256: G[i][j] += sum over voxel chunk blockIdx.x (csz voxels) of
// x[i][n] x[j][n] for the whole upper triangle, so that every sample is
// staged once.  Stage: 32 voxels of all frames in LDS (rows padded to 36
// floats: the 16-byte fragment reads of 16 rows fall in distinct banks).
// The triangle is cut into 32 x 32 super-tiles (I, J), I <= J; wavefront w
// owns super-rows w and 7 - w, nine super-tiles, each 2 x 2 MFMA tiles of
// v_mfma_f32_16x16x4_f32.  A lane reads four consecutive voxels of its row
// (one b128) and feeds them to four MFMAs: the contracted index of MFMA c is
// voxel 4 (lane / 16) + c of the 16-voxel half-stage, the same for both
// operands, so the sum runs over every voxel once.
constexpr int kFullT = 256;
constexpr int GF_KV = 32;
constexpr int GF_PITCH = GF_KV + 4;

__global__ __launch_bounds__(256) void gram_full(const float* __restrict__ x, int T, long long N,
                                                 long long csz, double* __restrict__ G) {
  __shared__ __attribute__((aligned(16))) float Xs[kFullT * GF_PITCH];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int ng = (T + 31) >> 5;  // super-rows
  const int rows = 32 * ng;
  const long long v0 = (long long)blockIdx.x * csz;
  const long long v1 = min(N, v0 + csz);
  const bool vec = (N & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
  f32x4 acc[9][2][2];
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) acc[q][u][v] = f32x4{0.f, 0.f, 0.f, 0.f};
  // the next stage's samples are loaded into registers while the MFMAs of
  // the current one run (one wavefront per SIMD: nothing else hides them)
  constexpr int kQuads = kFullT * GF_KV / 4 / 256;  // 16-byte loads per thread
  f32x4 pre[kQuads];
  auto fetch = [&](long long s) {
    const bool full = vec && s + GF_KV <= v1;
#pragma unroll
    for (int i = 0; i < kQuads; ++i) {
      const int idx = t + 256 * i, r = idx >> 3, qd = idx & 7;
      f32x4 val = f32x4{0.f, 0.f, 0.f, 0.f};
      if (r < T) {
        const float* src = x + (long long)r * N + s + 4 * qd;
        if (full) {
          val = *reinterpret_cast<const f32x4*>(src);
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (s + 4 * qd + c < v1) val[c] = src[c];
        }
      }
      pre[i] = val;
    }
  };
  if (v0 < v1) fetch(v0);
  for (long long s = v0; s < v1; s += GF_KV) {
    __syncthreads();  // the previous stage is no longer read
#pragma unroll
    for (int i = 0; i < kQuads; ++i) {
      const int idx = t + 256 * i, r = idx >> 3, qd = idx & 7;
      if (r < rows) *reinterpret_cast<f32x4*>(Xs + r * GF_PITCH + 4 * qd) = pre[i];
    }
    __syncthreads();
    if (s + GF_KV < v1) fetch(s + GF_KV);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = 16 * h + 4 * (lane >> 4);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        // super-tile q of this wavefront
        const int I = q <= 7 - wave ? wave : 7 - wave;
        const int J = q <= 7 - wave ? wave + q : q - 1;
        if (J >= ng) continue;  // uniform over the wavefront
        f32x4 a[2], b[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          a[u] = *reinterpret_cast<const f32x4*>(Xs + (32 * I + 16 * u + (lane & 15)) * GF_PITCH + col);
          b[u] = *reinterpret_cast<const f32x4*>(Xs + (32 * J + 16 * u + (lane & 15)) * GF_PITCH + col);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v)
              acc[q][u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][c], b[v][c], acc[q][u][v], 0, 0, 0);
      }
    }
  }
  // D of a tile: lane holds rows 4 (lane / 16) + r, column lane % 16
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int I = q <= 7 - wave ? wave : 7 - wave;
    const int J = q <= 7 - wave ? wave + q : q - 1;
    if (J >= ng) continue;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 32 * I + 16 * u + 4 * (lane >> 4) + r;
          const int j = 32 * J + 16 * v + (lane & 15);
          if (j < T && i <= j) atomicAdd(G + (size_t)i * T + j, (double)acc[q][u][v][r]);
        }
  }
}

constexpr int kMaxT = 512;

// Block-wide FP64 sum over blockDim.x threads (a multiple of 64, at most
// 1024); every thread returns the total.  red: 16 doubles of LDS.
__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int nw = blockDim.x >> 6;
  __syncthreads();  // red is free (a previous call has been read)
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += red[w];
  return t;
}

// ---------------------------------------------------------------------------
// Eigen-decomposition of the FP64 Gram matrix G (T x T, T <= 512) in four
// steps, all in FP64:
//   1. Householder reduction to tridiagonal form, Q^T G Q = tridiag(e, d, e),
//      Q = H_0 H_1 ... H_{T-3}, H_k = I - tau_k u_k u_k^T (one workgroup; the
//      working matrix lives in global memory and stays in L2);
//   2. every eigenvalue of the tridiagonal matrix by multisection on Sturm
//      counts (one wavefront per eigenvalue, 64 points per iteration);
//   3. the eigenvectors of the projection basis by inverse iteration (one
//      wavefront per vector, LU with partial pivoting of the shifted
//      tridiagonal matrix in LDS), re-orthogonalised within clusters of
//      (nearly) equal eigenvalues;
//   4. back-transformation V = Q Y (one workgroup per vector).
// FP64 keeps every eigenvector accurate to ~1e-16 of the largest eigenvalue
// over its gap, also for the weak components of a wide dynamic range.

// 1. A: working copy of G (full, row-major, mirrored from the upper triangle
// that the Gram kernel forms); on return row k right of the diagonal holds
// the Householder vector u_k (entries k+1 .. T-1).  Column k of the symmetric
// working matrix is read as row k, and u_k written there, so both are
// contiguous.
//
// Blocked by panels of kPanel columns: within a panel the trailing matrix is
// not touched; column k and the product B u_k are corrected on the fly for
// the panel's earlier reflectors (B_cur = B - V W^T - W V^T, with V the
// panel's Householder vectors and W the vectors w_k of their symmetric rank-2
// updates), and the whole trailing matrix takes one rank-2 kPanel update at
// the end of the panel: one read and write of it per panel instead of per
// column.  V and W live in LDS (dynamic, 2 T kPanel doubles).  Threads:
// (row quarter, column) for the matrix passes, so consecutive threads read
// consecutive addresses of a row; B is symmetric, so p_c = sum_r B[r][c] u_r.
constexpr int kPanel = 8;

__global__ __launch_bounds__(1024) void tri_reduce(const double* __restrict__ G, int T,
                                                   double* __restrict__ A, double* __restrict__ d,
                                                   double* __restrict__ e, double* __restrict__ tau) {
  extern __shared__ double panel[];  // Vp[T][kPanel], Wp[T][kPanel]
  __shared__ double u[kMaxT], wv[kMaxT], pp[4 * kMaxT], red[16], ycor[2 * kPanel * 2], x0s;
  double* Vp = panel;
  double* Wp = panel + (size_t)T * kPanel;
  const int tid = threadIdx.x, col = tid & 255, part = tid >> 8;  // blockDim.x = 1024
  // G holds the upper triangle (the Gram kernel forms blocks I <= J)
  for (int w = tid; w < T * T; w += blockDim.x) {
    const int i = w / T, j = w - i * T;
    A[w] = i <= j ? G[w] : G[(size_t)j * T + i];
  }
  for (int k0 = 0; k0 + 2 < T;) {
    const int npn = min(kPanel, T - 2 - k0);
    __syncthreads();  // A mirrored / the previous panel's update no longer reads V, W
    for (int w = tid; w < 2 * T * kPanel; w += blockDim.x) panel[w] = 0.0;
    __syncthreads();  // panel cleared; the previous update's writes to A done
    for (int i = 0; i < npn; ++i) {
      const int k = k0 + i;
      const int n = T - k - 1;  // the trailing block is rows / columns k+1 .. T-1
      // column k, rows k .. T-1 (read as row k: the panel's start matrix is
      // symmetric and row k is not written before), with the panel's earlier
      // reflectors applied
      double a = 0.0;
      if (tid <= n) {
        const int r = k + tid;
        a = A[(size_t)k * T + r];
        for (int j = 0; j < i; ++j)
          a -= Vp[r * kPanel + j] * Wp[k * kPanel + j] + Wp[r * kPanel + j] * Vp[k * kPanel + j];
        if (tid >= 1) u[tid - 1] = a;
        if (tid == 1) x0s = a;  // its own slot: thread 0 rewrites u[0] below
      }
      const double ss = block_sum(tid >= 1 && tid <= n ? a * a : 0.0, red);  // u, x0s visible after
      const double x0 = x0s;
      const double tail = ss - x0 * x0;
      if (tail <= 1e-300 * fmax(ss, 1e-300) || ss == 0.0) {
        // column already reduced: H_k = I (its V and W columns stay zero)
        if (tid == 0) {
          d[k] = a;
          e[k] = x0;
          tau[k] = 0.0;
        }
        __syncthreads();
        continue;
      }
      const double alpha = x0 >= 0.0 ? -sqrt(ss) : sqrt(ss);
      const double t = 1.0 / (alpha * (alpha - x0));  // 2 / (u^T u)
      if (tid == 0) {
        u[0] = x0 - alpha;
        d[k] = a;
        e[k] = alpha;
        tau[k] = t;
      }
      __syncthreads();
      // B u with the trailing matrix as it stood at the panel's start
      const int r0 = part * ((n + 3) >> 2), r1 = min(n, r0 + ((n + 3) >> 2));
      for (int c = col; c < n; c += 256) {
        const double* bc = A + (size_t)(k + 1) * T + (k + 1) + c;
        double acc = 0.0;
#pragma unroll 4
        for (int r = r0; r < r1; ++r) acc += bc[(size_t)r * T] * u[r];
        pp[part * kMaxT + c] = acc;
      }
      // y1 = W^T u, y2 = V^T u over rows k+1 .. T-1 (panel columns j < i):
      // two wavefronts per column j, lanes striding over the rows
      if (i > 0) {
        const int j = tid >> 7, h = tid & 127;
        double s1 = 0.0, s2 = 0.0;
        if (j < i)
          for (int r = h; r < n; r += 128) {
            s1 += Wp[(k + 1 + r) * kPanel + j] * u[r];
            s2 += Vp[(k + 1 + r) * kPanel + j] * u[r];
          }
        for (int o = 32; o > 0; o >>= 1) {
          s1 += __shfl_xor(s1, o);
          s2 += __shfl_xor(s2, o);
        }
        if ((tid & 63) == 0 && j < i) {
          ycor[(j * 2 + (h >> 6)) * 2] = s1;
          ycor[(j * 2 + (h >> 6)) * 2 + 1] = s2;
        }
      }
      __syncthreads();
      // p = t (B u - V y1 - W y2)
      if (tid < n) {
        double p = pp[tid] + pp[kMaxT + tid] + pp[2 * kMaxT + tid] + pp[3 * kMaxT + tid];
        const int r = k + 1 + tid;
        for (int j = 0; j < i; ++j) {
          const double y1 = ycor[(j * 2) * 2] + ycor[(j * 2 + 1) * 2];
          const double y2 = ycor[(j * 2) * 2 + 1] + ycor[(j * 2 + 1) * 2 + 1];
          p -= Vp[r * kPanel + j] * y1 + Wp[r * kPanel + j] * y2;
        }
        wv[tid] = t * p;
      }
      // w = p - (t/2 u^T p) u
      const double up_ = block_sum(tid < n ? u[tid] * wv[tid] : 0.0, red);
      const double K = 0.5 * t * up_;
      if (tid < n) {
        const double w = wv[tid] - K * u[tid];
        const int r = k + 1 + tid;
        Vp[r * kPanel + i] = u[tid];
        Wp[r * kPanel + i] = w;
        A[(size_t)k * T + r] = u[tid];
      }
      __syncthreads();
    }
    // trailing rows / columns s0 .. T-1: B -= V W^T + W V^T (the panel's
    // columns of W and V for column c held in registers)
    const int s0 = k0 + npn, m = T - s0;
    const int r0 = part * ((m + 3) >> 2), r1 = min(m, r0 + ((m + 3) >> 2));
    for (int c = s0 + col; c < T; c += 256) {
      double wc[kPanel], vc[kPanel];
#pragma unroll
      for (int j = 0; j < kPanel; ++j) {
        wc[j] = Wp[c * kPanel + j];
        vc[j] = Vp[c * kPanel + j];
      }
      for (int r = s0 + r0; r < s0 + r1; ++r) {
        double* ar = A + (size_t)r * T + c;
        double acc = *ar;
#pragma unroll
        for (int j = 0; j < kPanel; ++j) acc -= Vp[r * kPanel + j] * wc[j] + Wp[r * kPanel + j] * vc[j];
        *ar = acc;
      }
    }
    k0 += npn;
  }
  __syncthreads();
  if (tid == 0) {
    if (T >= 2) {
      d[T - 2] = A[(size_t)(T - 2) * T + T - 2];
      e[T - 2] = A[(size_t)(T - 1) * T + T - 2];
      tau[T - 2] = 0.0;
    }
    d[T - 1] = A[(size_t)(T - 1) * T + T - 1];
    if (T >= 1) tau[T - 1] = 0.0;
  }
}

size_t tri_reduce_lds(int T) { return 2 * sizeof(double) * (size_t)T * kPanel; }

// Number of eigenvalues of tridiag(e, d, e) below x (Sturm sequence of the
// LDL^T factorisation of T - x I; zero pivots replaced by -pivmin).
__device__ inline int sturm_count(const double* d, const double* e2, int T, double x, double pivmin) {
  double q = d[0] - x;
  int c = q < 0.0;
  for (int t = 1; t < T; ++t) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = d[t] - x - e2[t - 1] / q;
    c += q < 0.0;
  }
  return c;
}

// 2. Eigenvalue i (ascending) in wavefront i: 64 points per iteration, the
// bracket shrinks 65-fold each time; Gershgorin bounds to start.
__global__ __launch_bounds__(64) void tri_bisect(const double* __restrict__ d,
                                                 const double* __restrict__ e, int T,
                                                 double* __restrict__ lam) {
  __shared__ double sd[kMaxT], se2[kMaxT];
  const int lane = threadIdx.x, i = blockIdx.x;
  double lo = 1e300, hi = -1e300, emax = 0.0;
  for (int t = lane; t < T; t += 64) {
    const double el = t > 0 ? fabs(e[t - 1]) : 0.0, er = t + 1 < T ? fabs(e[t]) : 0.0;
    sd[t] = d[t];
    se2[t] = er * er;
    lo = fmin(lo, d[t] - el - er);
    hi = fmax(hi, d[t] + el + er);
    emax = fmax(emax, er);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
    emax = fmax(emax, __shfl_xor(emax, o));
  }
  __syncthreads();
  const double scale = fmax(fabs(lo), fabs(hi));
  const double pivmin = fmax(1e-290, 1e-300 * emax * emax);
  lo -= 1e-14 * scale + 1e-300;
  hi += 1e-14 * scale + 1e-300;
  for (int it = 0; it < 12 && hi - lo > 2e-16 * fmax(fabs(lo), fabs(hi)); ++it) {
    const double h = (hi - lo) / 65.0;
    const double x = lo + (lane + 1) * h;
    const int c = sturm_count(sd, se2, T, x, pivmin);
    // first point with more than i eigenvalues below it
    const uint64_t above = __ballot(c > i);
    const int j = above ? __builtin_ctzll(above) : 64;
    const double nlo = lo + j * h, nhi = j < 64 ? lo + (j + 1) * h : hi;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) lam[i] = 0.5 * (lo + hi);
}

// Rank of eigenvalue i in descending order, ties by index (the order the
// filter's component numbers k_lo, k_hi refer to).
__device__ inline int descending_rank(const double* lam, int T, int i) {
  const double li = lam[i];
  int rk = 0;
  for (int j = 0; j < T; ++j) {
    const double lj = lam[j];
    rk += (lj > li) || (lj == li && j < i);
  }
  return rk;
}

// Whether eigenvalue i's eigenvector enters the projection basis: the
// components k_lo .. k_hi-1 (keep form) or the others (removal form).
__device__ inline bool in_projection_basis(const double* lam, int T, int i, int k_lo, int k_hi,
                                           int keep) {
  const int rk = descending_rank(lam, T, i);
  const bool band = rk >= k_lo && rk < k_hi;
  return keep ? band : !band;
}

// 3. Inverse iteration for the eigenvectors of the projection basis (the
// others are never used), one workgroup of one wavefront per eigenvector j:
// the wavefront copies the tridiagonal matrix to LDS, then lane 0 does the
// serial work there: Gaussian elimination with
// partial pivoting of tridiag(e, d, e) - lam_j I (U with two
// superdiagonals, multipliers and row-swap flags), then three solves from a
// fixed pseudo-random start, each normalised.  Y[t][j] = component t.
__global__ __launch_bounds__(64) void tri_inverse(const double* __restrict__ d,
                                                  const double* __restrict__ e,
                                                  const double* __restrict__ lam, int T, int k_lo,
                                                  int k_hi, int keep, double* __restrict__ Y) {
  __shared__ double U0[kMaxT], U1[kMaxT], U2[kMaxT], L[kMaxT], y[kMaxT], sd[kMaxT], se[kMaxT];
  __shared__ unsigned char P[kMaxT];
  const int j = blockIdx.x;
  if (!in_projection_basis(lam, T, j, k_lo, k_hi, keep)) return;  // uniform
  // the tridiagonal matrix in LDS (the wavefront), then lane 0 alone
  double anorm = 0.0;
  for (int t = threadIdx.x; t < T; t += blockDim.x) {
    sd[t] = d[t];
    se[t] = e[t];
    anorm = fmax(anorm, fabs(d[t]) + (t > 0 ? fabs(e[t - 1]) : 0.0) + (t + 1 < T ? fabs(e[t]) : 0.0));
  }
  for (int o = 32; o > 0; o >>= 1) anorm = fmax(anorm, __shfl_xor(anorm, o));
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double tiny = fmax(1e-280, 2.2e-16 * anorm);
  const double lj = lam[j];
  // the current row has entries (a, b) at (x_t, x_{t+1}); the next original
  // row is (e_t, d_{t+1} - lam, e_{t+1}) at (x_t, x_{t+1}, x_{t+2})
  double a = sd[0] - lj, b = T > 1 ? se[0] : 0.0;
  for (int t = 0; t + 1 < T; ++t) {
    const double sub = se[t], na = sd[t + 1] - lj, nb = t + 2 < T ? se[t + 1] : 0.0;
    if (fabs(sub) > fabs(a)) {  // swap: the next row is the pivot row
      const double m = a / sub;
      U0[t] = sub;
      U1[t] = na;
      U2[t] = nb;
      L[t] = m;
      P[t] = 1;
      a = b - m * na;
      b = -m * nb;
    } else {
      if (fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
      const double m = sub / a;
      U0[t] = a;
      U1[t] = b;
      U2[t] = 0.0;
      L[t] = m;
      P[t] = 0;
      a = na - m * b;
      b = nb;
    }
  }
  if (fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
  U0[T - 1] = a;
  U1[T - 1] = 0.0;
  U2[T - 1] = 0.0;
  // start vector
  for (int t = 0; t < T; ++t) {
    const uint32_t h = (uint32_t)t * 2654435761u ^ ((uint32_t)j * 40503u + 0x9e3779b9u);
    y[t] = 0.5 + (double)((h >> 8) & 0xffff) / 65536.0;
  }
  for (int it = 0; it < 3; ++it) {
    // forward: apply the row operations to the right-hand side (in place)
    double r = y[0];
    for (int t = 0; t + 1 < T; ++t) {
      const double y1 = y[t + 1], m = L[t];
      if (P[t]) {
        y[t] = y1;
        r = r - m * y1;
      } else {
        y[t] = r;
        r = y1 - m * r;
      }
    }
    y[T - 1] = r;
    // back substitution
    double x2 = 0.0, x1 = y[T - 1] / U0[T - 1];
    y[T - 1] = x1;
    double nrm = x1 * x1;
    for (int t = T - 2; t >= 0; --t) {
      const double x = (y[t] - U1[t] * x1 - U2[t] * x2) / U0[t];
      y[t] = x;
      nrm += x * x;
      x2 = x1;
      x1 = x;
    }
    const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
    for (int t = 0; t < T; ++t) y[t] *= inv;
  }
  for (int t = 0; t < T; ++t) Y[(size_t)t * T + j] = y[t];
}

// 3b. Re-orthogonalise, within clusters of eigenvalues closer than 1e-9 of
// the spectral radius, the eigenvectors that enter the projection basis
// (inverse iteration leaves vectors of (nearly) equal eigenvalues
// non-orthogonal): classical Gram-Schmidt applied twice, in ascending order,
// each basis vector against the cluster's earlier basis vectors.  The other
// eigenvectors are never used, so they are left as they are; one workgroup.
__global__ __launch_bounds__(1024) void tri_orth(const double* __restrict__ lam, int T, int k_lo,
                                                 int k_hi, int keep, double* __restrict__ Y) {
  __shared__ double dots[kMaxT], ls[kMaxT], red[16];
  __shared__ int in_basis[kMaxT];
  const int tid = threadIdx.x;
  double lmax = 0.0;
  for (int i = tid; i < T; i += blockDim.x) {
    in_basis[i] = in_projection_basis(lam, T, i, k_lo, k_hi, keep);
    ls[i] = lam[i];
    lmax = fmax(lmax, fabs(lam[i]));
  }
  for (int o = 32; o > 0; o >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, o));
  if ((tid & 63) == 0) red[tid >> 6] = lmax;
  __syncthreads();
  lmax = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) lmax = fmax(lmax, red[w]);
  __syncthreads();  // red is reused by block_sum below
  const double tol = 1e-9 * lmax;
  int cs = 0;  // first vector of the current cluster
  for (int j = 1; j < T; ++j) {
    if (ls[j] - ls[j - 1] > tol) {
      cs = j;
      continue;
    }
    if (!in_basis[j]) continue;  // uniform over the workgroup
    for (int pass = 0; pass < 2; ++pass) {
      // dots with the cluster's earlier basis vectors (one thread each)
      for (int i = cs + tid; i < j; i += blockDim.x) {
        double acc = 0.0;
        if (in_basis[i])  // other columns of Y are not formed
          for (int t = 0; t < T; ++t) acc += Y[(size_t)t * T + i] * Y[(size_t)t * T + j];
        dots[i] = acc;
      }
      __syncthreads();
      for (int t = tid; t < T; t += blockDim.x) {
        double y = Y[(size_t)t * T + j];
        for (int i = cs; i < j; ++i)
          if (in_basis[i]) y -= dots[i] * Y[(size_t)t * T + i];
        Y[(size_t)t * T + j] = y;
      }
      __syncthreads();
    }
    double part = 0.0;
    for (int t = tid; t < T; t += blockDim.x) part += Y[(size_t)t * T + j] * Y[(size_t)t * T + j];
    const double nrm = block_sum(part, red);
    const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
    for (int t = tid; t < T; t += blockDim.x) Y[(size_t)t * T + j] *= inv;
    __syncthreads();
  }
}

// 4. V = Q Y for the basis eigenvectors, one wavefront per eigenvector j:
// the Householder reflectors H_{T-3} .. H_0 applied in turn (u_k read from
// row k, tau from LDS).  Each step is a dot product and an update over at
// most T - 1 entries.  The vector stays in registers (entry c in lane c mod
// 64), so a step is a few LDS reads of u_k, FMAs and one shuffle reduction;
// the rows are staged in LDS a chunk of 5120 / T rows at a time with all of
// a chunk's loads in flight together.
__global__ __launch_bounds__(64) void tri_back(const double* __restrict__ A,
                                               const double* __restrict__ tau,
                                               const double* __restrict__ Y,
                                               const double* __restrict__ lam, int T, int k_lo,
                                               int k_hi, int keep, double* __restrict__ V) {
  constexpr int BUF = 5120;      // staged row entries (40 KiB)
  constexpr int R = kMaxT / 64;  // vector entries per lane
  __shared__ double ts[kMaxT], ub[BUF];
  const int j = blockIdx.x, lane = threadIdx.x;
  if (!in_projection_basis(lam, T, j, k_lo, k_hi, keep)) return;  // uniform
  double y[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int c = lane + 64 * r;
    y[r] = c < T ? Y[(size_t)c * T + j] : 0.0;
  }
  for (int t = lane; t < T; t += 64) ts[t] = tau[t];
  const int rows = BUF / T;  // >= 10 for T <= 512
  for (int khi = T - 3; khi >= 0; khi -= rows) {
    const int klo = max(khi - rows + 1, 0);
    __syncthreads();  // the previous chunk's reads are done
    // row k, entries k+1 .. T-1, to ub[(khi - k) T + column]: the chunk as
    // one flat range, 32 loads per lane issued before their LDS stores
    const int span = (khi - klo + 1) * T;
    for (int base = 0; base < span; base += 64 * 32) {
      double v[32];
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const int idx = base + m * 64 + lane;
        const int rr = idx / T, c = idx - rr * T, k = khi - rr;
        v[m] = (idx < span && c > k) ? A[(size_t)k * T + c] : 0.0;
      }
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const int idx = base + m * 64 + lane;
        if (idx < span) ub[idx] = v[m];
      }
    }
    __syncthreads();
    for (int k = khi; k >= klo; --k) {
      const double tk = ts[k];
      if (tk == 0.0) continue;  // uniform
      const double* u = ub + (size_t)(khi - k) * T;
      double uk[R], part = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int c = lane + 64 * r;
        uk[r] = (c > k && c < T) ? u[c] : 0.0;  // u_k is zero at and above k
        part = fma(uk[r], y[r], part);
      }
      for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
      const double sc = tk * part;
#pragma unroll
      for (int r = 0; r < R; ++r) y[r] = fma(-sc, uk[r], y[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int c = lane + 64 * r;
    if (c < T) V[(size_t)c * T + j] = y[r];
  }
}

// Rank the eigenvalues (descending, ties by index), write sigma = sqrt(lambda),
// and copy the projection basis B[T][nb] (FP32 and FP64): the eigenvectors of
// ranks [k_lo, k_hi) for the keep form, the others for the removal form.
__global__ __launch_bounds__(1024) void rank_basis(const double* __restrict__ lam,
                                                   const double* __restrict__ v, int T, int k_lo,
                                                   int k_hi, int keep, float* __restrict__ sv,
                                                   float* __restrict__ Bm, double* __restrict__ Bd,
                                                   int nb) {
  __shared__ int rank_of[kMaxT];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < T; i += nt) {
    const int rk = descending_rank(lam, T, i);
    rank_of[rk] = i;
    sv[rk] = (float)sqrt(fmax(lam[i], 0.0));
  }
  __syncthreads();
  for (int w = tid; w < T * nb; w += nt) {
    const int t = w / nb, j = w - t * nb;
    const int rk = keep ? k_lo + j : (j < k_lo ? j : k_hi + (j - k_lo));
    const double b = v[(size_t)t * T + rank_of[rk]];
    Bm[w] = (float)b;
    Bd[w] = b;
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

// Power only (no filtered series): with B orthonormal, a = B^T s_n carries
// the kept energy |a|^2 (keep form), and the removal form keeps
// |s_n|^2 - |a|^2; both in FP64 with the FP64 basis, so the difference is
// exact to far below the FP32 output even when the removed clutter is many
// orders above the rest.  One read of the series, one voxel per thread (the
// form for 5 to 16 basis vectors; smaller bases take power_split below).
// NBMAX >= nb.
template <int NBMAX>
__global__ __launch_bounds__(256) void power_1pass(const float* __restrict__ x, int T, long long N,
                                                   const double* __restrict__ Bd, int nb, int keep,
                                                   float* __restrict__ pd) {
  extern __shared__ double Bs64[];
  for (int i = threadIdx.x; i < T * nb; i += blockDim.x) Bs64[i] = Bd[i];
  __syncthreads();
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double a[NBMAX], ss = 0.0;
#pragma unroll
  for (int j = 0; j < NBMAX; ++j) a[j] = 0.0;
#pragma unroll 4
  for (int t = 0; t < T; ++t) {
    const double sv = (double)x[(long long)t * N + n];
    ss = fma(sv, sv, ss);
#pragma unroll
    for (int j = 0; j < NBMAX; ++j)
      if (j < nb) a[j] = fma(sv, Bs64[t * nb + j], a[j]);
  }
  double aa = 0.0;
#pragma unroll
  for (int j = 0; j < NBMAX; ++j) aa = fma(a[j], a[j], aa);
  const double p = keep ? aa : fmax(ss - aa, 0.0);
  pd[n] = (float)(p / T);
}

// The same one-pass power for small bases (nb <= 4) with the frames split
// over the four wavefronts of a workgroup: each wavefront sums a quarter of
// the frames for the block's 256 voxels (four neighbouring voxels per lane,
// one 16-byte load per frame), then the partial sums (FP64) are added in LDS
// in two pairwise rounds.  Four times the wavefronts of the voxel-per-thread
// form for the same ensemble: more loads in flight and a short tail.
template <int NBMAX>
__global__ __launch_bounds__(256) void power_split(const float* __restrict__ x, int T, long long N,
                                                   const double* __restrict__ Bd, int nb, int keep,
                                                   float* __restrict__ pd) {
  constexpr int VPT = 4, NV = NBMAX + 1, R = VPT * NV;  // partial sums per lane
  extern __shared__ double Bs64[];                       // [T nb] basis, then [2][R][64] partials
  double* const red = Bs64 + ((T * nb + 1) & ~1);
  for (int i = threadIdx.x; i < T * nb; i += blockDim.x) Bs64[i] = Bd[i];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long n0 = ((long long)blockIdx.x * 64 + lane) * VPT;
  const bool full = n0 + VPT <= N && (N & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
  double part[R];  // [v][0] = sum s^2, [v][1 + j] = sum s B_j
#pragma unroll
  for (int i = 0; i < R; ++i) part[i] = 0.0;
  if (n0 < N) {
    const int tb = T * wave / 4, te = T * (wave + 1) / 4;
#pragma unroll 4
    for (int t = tb; t < te; ++t) {
      const float* row = x + (long long)t * N + n0;
      float sv[VPT];
      if (full) {
        const f32x4 q = *reinterpret_cast<const f32x4*>(row);
#pragma unroll
        for (int v = 0; v < VPT; ++v) sv[v] = q[v];
      } else {
#pragma unroll
        for (int v = 0; v < VPT; ++v) sv[v] = n0 + v < N ? row[v] : 0.f;
      }
#pragma unroll
      for (int v = 0; v < VPT; ++v) {
        const double d = (double)sv[v];
        part[v * NV] = fma(d, d, part[v * NV]);
#pragma unroll
        for (int j = 0; j < NBMAX; ++j)
          if (j < nb) part[v * NV + 1 + j] = fma(d, Bs64[t * nb + j], part[v * NV + 1 + j]);
      }
    }
  }
  // waves 2, 3 hand their sums to waves 0, 1; then wave 1 to wave 0
  // (every wave reaches every barrier)
  if (wave >= 2) {
#pragma unroll
    for (int i = 0; i < R; ++i) red[((wave - 2) * R + i) * 64 + lane] = part[i];
  }
  __syncthreads();
  if (wave < 2) {
#pragma unroll
    for (int i = 0; i < R; ++i) part[i] += red[(wave * R + i) * 64 + lane];
  }
  __syncthreads();
  if (wave == 1) {
#pragma unroll
    for (int i = 0; i < R; ++i) red[i * 64 + lane] = part[i];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int v = 0; v < VPT; ++v) {
    if (n0 + v >= N) break;
    double aa = 0.0;
#pragma unroll
    for (int j = 0; j < NBMAX; ++j) {
      const double aj = part[v * NV + 1 + j] + red[(v * NV + 1 + j) * 64 + lane];
      aa = fma(aj, aj, aa);
    }
    const double ss = part[v * NV] + red[(v * NV) * 64 + lane];
    const double p = keep ? aa : fmax(ss - aa, 0.0);
    pd[n0 + v] = (float)(p / T);
  }
}

hipError_t launch_power_split(const float* x, int T, long long N, const double* Bd, int nb, int keep,
                              float* pd, hipStream_t st) {
  constexpr int NBMAX = 4, R = 4 * (NBMAX + 1);
  const size_t lds = sizeof(double) * ((size_t)((T * nb + 1) & ~1) + 2 * R * 64);
  hipLaunchKernelGGL((power_split<NBMAX>), dim3((unsigned)((N + 255) / 256)), dim3(256), lds, st, x,
                     T, N, Bd, nb, keep, pd);
  return hipGetLastError();
}

template <int NBMAX>
hipError_t launch_power_1pass(const float* x, int T, long long N, const double* Bd, int nb, int keep,
                              float* pd, hipStream_t st) {
  const size_t lds = sizeof(double) * (size_t)T * nb;
  hipLaunchKernelGGL((power_1pass<NBMAX>), dim3((unsigned)((N + 255) / 256)), dim3(256), lds, st, x,
                     T, N, Bd, nb, keep, pd);
  return hipGetLastError();
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

// Workspace layout (bytes from the start), every part 256-byte aligned:
// G, V, A, Y (T x T f64 each), Bm (T x 64 f32), Bd (T x 64 f64), d, e, tau,
// lam (T f64 each).
struct ClutterWs {
  size_t G, V, A, Y, Bm, Bd, d, e, tau, lam, total;
};
constexpr ClutterWs ws_layout(int T) {
  const size_t tt = align256(sizeof(double) * (size_t)T * T), t8 = align256(sizeof(double) * (size_t)T);
  ClutterWs L{};
  size_t o = 0;
  L.G = o; o += tt;
  L.V = o; o += tt;
  L.A = o; o += tt;
  L.Y = o; o += tt;
  L.Bm = o; o += align256(sizeof(float) * (size_t)T * 64);
  L.Bd = o; o += align256(sizeof(double) * (size_t)T * 64);
  L.d = o; o += t8;
  L.e = o; o += t8;
  L.tau = o; o += t8;
  L.lam = o; o += t8;
  L.total = o;
  return L;
}
constexpr size_t workspace_bytes(int T) { return ws_layout(T).total; }

// Workspace of the allocation-free entry point: room for ensembles of up to
// kStaticT frames (2.2 MiB), one copy per device, held until the process
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
  const ClutterWs L = ws_layout(T);
  double* G = reinterpret_cast<double*>(w + L.G);
  double* V = reinterpret_cast<double*>(w + L.V);
  double* A = reinterpret_cast<double*>(w + L.A);
  double* Y = reinterpret_cast<double*>(w + L.Y);
  float* Bm = reinterpret_cast<float*>(w + L.Bm);
  double* Bd = reinterpret_cast<double*>(w + L.Bd);
  double* d = reinterpret_cast<double*>(w + L.d);
  double* e_ = reinterpret_cast<double*>(w + L.e);
  double* tau = reinterpret_cast<double*>(w + L.tau);
  double* lam = reinterpret_cast<double*>(w + L.lam);
  const int kept = k_hi - k_lo;
  const int keep = kept <= T - kept ? 1 : 0;
  const int nb = keep ? kept : T - kept;
  hipLaunchKernelGGL(zero_f64, dim3(256), dim3(256), 0, st, G, (size_t)T * T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (T <= kFullT) {
    // two workgroups per CU, each a whole number of 32-voxel stages
    const long long nstage = (N + GF_KV - 1) / GF_KV;
    const long long nwg = std::max(1LL, std::min(nstage, 2LL * cus));
    const long long csz = (nstage + nwg - 1) / nwg * GF_KV;
    const long long nch = (N + csz - 1) / csz;
    hipLaunchKernelGGL(gram_full, dim3((unsigned)nch), dim3(256), 0, st, x, T, N, csz, G);
  } else {
    const int nbk = (T + GB - 1) / GB, npairs = nbk * (nbk + 1) / 2;
    const long long nsteps = (N + GB - 1) / GB;
    const long long nchunk = std::max(1LL, std::min(nsteps, (long long)(8 * cus) / npairs + 1));
    const long long csz = (nsteps + nchunk - 1) / nchunk * GB;
    const long long nch = (N + csz - 1) / csz;
    hipLaunchKernelGGL(gram_mfma, dim3((unsigned)npairs, (unsigned)nch), dim3(256), 0, st, x, T, N,
                       csz, nbk, G);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  {
    const size_t lds = tri_reduce_lds(T);
    if ((e = hipFuncSetAttribute((const void*)tri_reduce, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(tri_reduce, dim3(1), dim3(1024), lds, st, G, T, A, d, e_, tau);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tri_bisect, dim3(T), dim3(64), 0, st, d, e_, T, lam);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tri_inverse, dim3(T), dim3(64), 0, st, d, e_, lam, T, k_lo, k_hi, keep, Y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tri_orth, dim3(1), dim3(1024), 0, st, lam, T, k_lo, k_hi, keep, Y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tri_back, dim3(T), dim3(64), 0, st, A, tau, Y, lam, T, k_lo, k_hi, keep, V);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(rank_basis, dim3(1), dim3(1024), 0, st, lam, V, T, k_lo, k_hi, keep, sv, Bm, Bd,
                     nb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (!xf && nb > 0 && nb <= 16 && sizeof(double) * (size_t)T * nb <= 48 * 1024) {
    if (nb <= 4) return launch_power_split(x, T, N, Bd, nb, keep, pd, st);
    if (nb <= 8) return launch_power_1pass<8>(x, T, N, Bd, nb, keep, pd, st);
    return launch_power_1pass<16>(x, T, N, Bd, nb, keep, pd, st);
  }
  if (nb == 0) {  // keep nothing or remove nothing
    return launch_project<1>(x, T, N, Bm, 0, keep, pd, xf, st);
  }
  if (nb <= 8) return launch_project<8>(x, T, N, Bm, nb, keep, pd, xf, st);
  if (nb <= 16) return launch_project<16>(x, T, N, Bm, nb, keep, pd, xf, st);
  if (nb <= 32) return launch_project<32>(x, T, N, Bm, nb, keep, pd, xf, st);
  return launch_project<64>(x, T, N, Bm, nb, keep, pd, xf, st);
}

}  // namespace dasmi
