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
//   2. Eigen-decomposition G = V diag(lambda) V^T in FP64: Householder
//      tridiagonalisation (one workgroup, matrix in L2), all eigenvalues by
//      multisection on Sturm counts (one wavefront each), eigenvectors by
//      inverse iteration (one thread each) re-orthogonalised within
//      clusters, back-transformed by the reflectors (one workgroup each).
//      sigma = sqrt(lambda), sorted; the columns of V that the filter needs
//      are copied (FP32) as the projection basis B.
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
//   3. its eigenvectors by inverse iteration (one thread per vector, LU with
//      partial pivoting of the shifted tridiagonal matrix), re-orthogonalised
//      within clusters of (nearly) equal eigenvalues;
//   4. back-transformation V = Q Y (one workgroup per vector).
// FP64 keeps every eigenvector accurate to ~1e-16 of the largest eigenvalue
// over its gap, also for the weak components of a wide dynamic range.

// 1. A: working copy of G (full, row-major, mirrored from the upper triangle
// that the Gram kernel forms); on return column k below the diagonal holds
// the Householder vector u_k (entries k+1 .. T-1).
__global__ __launch_bounds__(1024) void tri_reduce(const double* __restrict__ G, int T,
                                                   double* __restrict__ A, double* __restrict__ d,
                                                   double* __restrict__ e, double* __restrict__ tau) {
  __shared__ double v[kMaxT], w[kMaxT], red[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  // G holds the upper triangle (the Gram kernel forms blocks I <= J)
  for (int w = tid; w < T * T; w += blockDim.x) {
    const int i = w / T, j = w - i * T;
    A[w] = i <= j ? G[w] : G[(size_t)j * T + i];
  }
  __syncthreads();
  for (int k = 0; k + 2 < T; ++k) {
    const int n = T - k - 1;  // the trailing block is rows / columns k+1 .. T-1
    const double xi = tid < n ? A[(size_t)(k + 1 + tid) * T + k] : 0.0;
    const double ss = block_sum(xi * xi, red);
    const double x0 = A[(size_t)(k + 1) * T + k];
    const double tail = ss - x0 * x0;
    if (tail <= 1e-300 * fmax(ss, 1e-300) || ss == 0.0) {
      // column already reduced: H_k = I
      if (tid == 0) {
        d[k] = A[(size_t)k * T + k];
        e[k] = x0;
        tau[k] = 0.0;
      }
      __syncthreads();
      continue;
    }
    const double alpha = x0 >= 0.0 ? -sqrt(ss) : sqrt(ss);
    const double t = 1.0 / (alpha * (alpha - x0));  // 2 / (u^T u)
    if (tid < n) v[tid] = tid == 0 ? x0 - alpha : xi;
    __syncthreads();
    // p = t B u (rows by wavefronts, columns by lanes), w = p - (t/2 u^T p) u
    for (int i = wave; i < n; i += nw) {
      const double* row = A + (size_t)(k + 1 + i) * T + (k + 1);
      double acc = 0.0;
      for (int j = lane; j < n; j += 64) acc += row[j] * v[j];
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      if (lane == 0) w[i] = t * acc;
    }
    __syncthreads();
    const double up_ = block_sum(tid < n ? v[tid] * w[tid] : 0.0, red);
    const double K = 0.5 * t * up_;
    if (tid < n) w[tid] -= K * v[tid];
    __syncthreads();
    // B -= u w^T + w u^T
    for (int i = wave; i < n; i += nw) {
      double* row = A + (size_t)(k + 1 + i) * T + (k + 1);
      const double vi = v[i], wi = w[i];
      for (int j = lane; j < n; j += 64) row[j] -= vi * w[j] + wi * v[j];
    }
    if (tid == 0) {
      d[k] = A[(size_t)k * T + k];
      e[k] = alpha;
      tau[k] = t;
    }
    if (tid < n) A[(size_t)(k + 1 + tid) * T + k] = v[tid];
    __syncthreads();
  }
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

// 3. Inverse iteration, one thread per eigenvector j: Gaussian elimination
// with partial pivoting of tridiag(e, d - lam_j, e) (U with two
// superdiagonals, multipliers and row-swap flags in sc[5][T][T], component-
// major so that the threads of a wavefront touch consecutive addresses),
// then three solves from a fixed pseudo-random start, each normalised.
// Y[t][j] = component t of eigenvector j.
__global__ __launch_bounds__(64) void tri_inverse(const double* __restrict__ d,
                                                  const double* __restrict__ e,
                                                  const double* __restrict__ lam, int T,
                                                  double* __restrict__ sc, double* __restrict__ Y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= T) return;
  const size_t TT = (size_t)T * T;
  double* U0 = sc;
  double* U1 = sc + TT;
  double* U2 = sc + 2 * TT;
  double* L = sc + 3 * TT;
  double* P = sc + 4 * TT;
  auto at = [&](double* arr, int t) -> double& { return arr[(size_t)t * T + j]; };
  double anorm = 0.0;
  for (int t = 0; t < T; ++t)
    anorm = fmax(anorm, fabs(d[t]) + (t > 0 ? fabs(e[t - 1]) : 0.0) + (t + 1 < T ? fabs(e[t]) : 0.0));
  const double tiny = fmax(1e-280, 2.2e-16 * anorm);
  const double lj = lam[j];
  // the current row has entries (a, b) at (x_t, x_{t+1}); the next original
  // row is (e_t, d_{t+1} - lam, e_{t+1}) at (x_t, x_{t+1}, x_{t+2})
  double a = d[0] - lj, b = T > 1 ? e[0] : 0.0;
  for (int t = 0; t + 1 < T; ++t) {
    const double sub = e[t], na = d[t + 1] - lj, nb = t + 2 < T ? e[t + 1] : 0.0;
    if (fabs(sub) > fabs(a)) {  // swap: the next row is the pivot row
      const double m = a / sub;
      at(U0, t) = sub;
      at(U1, t) = na;
      at(U2, t) = nb;
      at(L, t) = m;
      at(P, t) = 1.0;
      a = b - m * na;
      b = -m * nb;
    } else {
      if (fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
      const double m = sub / a;
      at(U0, t) = a;
      at(U1, t) = b;
      at(U2, t) = 0.0;
      at(L, t) = m;
      at(P, t) = 0.0;
      a = na - m * b;
      b = nb;
    }
  }
  if (fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
  at(U0, T - 1) = a;
  at(U1, T - 1) = 0.0;
  at(U2, T - 1) = 0.0;
  // start vector
  for (int t = 0; t < T; ++t) {
    const uint32_t h = (uint32_t)t * 2654435761u ^ ((uint32_t)j * 40503u + 0x9e3779b9u);
    at(Y, t) = 0.5 + (double)((h >> 8) & 0xffff) / 65536.0;
  }
  for (int it = 0; it < 3; ++it) {
    // forward: apply the row operations to the right-hand side (in place)
    double r = at(Y, 0);
    for (int t = 0; t + 1 < T; ++t) {
      const double y1 = at(Y, t + 1), m = at(L, t);
      if (at(P, t) != 0.0) {
        at(Y, t) = y1;
        r = r - m * y1;
      } else {
        at(Y, t) = r;
        r = y1 - m * r;
      }
    }
    at(Y, T - 1) = r;
    // back substitution
    double x2 = 0.0, x1 = at(Y, T - 1) / at(U0, T - 1);
    at(Y, T - 1) = x1;
    double nrm = x1 * x1;
    for (int t = T - 2; t >= 0; --t) {
      const double x = (at(Y, t) - at(U1, t) * x1 - at(U2, t) * x2) / at(U0, t);
      at(Y, t) = x;
      nrm += x * x;
      x2 = x1;
      x1 = x;
    }
    const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
    for (int t = 0; t < T; ++t) at(Y, t) *= inv;
  }
}

// 3b. Re-orthogonalise eigenvectors within clusters of eigenvalues closer
// than 1e-9 of the spectral radius (inverse iteration leaves vectors of
// (nearly) equal eigenvalues non-orthogonal), by classical Gram-Schmidt
// applied twice, in ascending order; one workgroup.
__global__ __launch_bounds__(1024) void tri_orth(const double* __restrict__ lam, int T,
                                                 double* __restrict__ Y) {
  __shared__ double dots[kMaxT], red[16];
  const int tid = threadIdx.x;
  double lmax = 0.0;
  for (int j = 0; j < T; ++j) lmax = fmax(lmax, fabs(lam[j]));
  const double tol = 1e-9 * lmax;
  int cs = 0;  // first vector of the current cluster
  for (int j = 1; j < T; ++j) {
    if (lam[j] - lam[j - 1] > tol) {
      cs = j;
      continue;
    }
    for (int pass = 0; pass < 2; ++pass) {
      // dots with the cluster's previous vectors (one thread each)
      for (int i = cs + tid; i < j; i += blockDim.x) {
        double acc = 0.0;
        for (int t = 0; t < T; ++t) acc += Y[(size_t)t * T + i] * Y[(size_t)t * T + j];
        dots[i] = acc;
      }
      __syncthreads();
      for (int t = tid; t < T; t += blockDim.x) {
        double y = Y[(size_t)t * T + j];
        for (int i = cs; i < j; ++i) y -= dots[i] * Y[(size_t)t * T + i];
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

// 4. V = Q Y, one workgroup per eigenvector j: the Householder reflectors
// H_{T-3} .. H_0 applied in turn.
__global__ __launch_bounds__(256) void tri_back(const double* __restrict__ A,
                                                const double* __restrict__ tau,
                                                const double* __restrict__ Y,
                                                int T, double* __restrict__ V) {
  __shared__ double y[kMaxT], red[16];
  const int j = blockIdx.x, tid = threadIdx.x;
  for (int t = tid; t < T; t += blockDim.x) y[t] = Y[(size_t)t * T + j];
  __syncthreads();
  for (int k = T - 3; k >= 0; --k) {
    const double tk = tau[k];
    if (tk == 0.0) continue;  // uniform
    const int n = T - k - 1;
    double part = 0.0;
    for (int i = tid; i < n; i += blockDim.x) part += A[(size_t)(k + 1 + i) * T + k] * y[k + 1 + i];
    const double s = tk * block_sum(part, red);
    for (int i = tid; i < n; i += blockDim.x) y[k + 1 + i] -= s * A[(size_t)(k + 1 + i) * T + k];
    __syncthreads();
  }
  for (int t = tid; t < T; t += blockDim.x) V[(size_t)t * T + j] = y[t];
}

// Rank the eigenvalues (descending, ties by index), write sigma = sqrt(lambda),
// and copy the projection basis B[T][nb] (FP32): the eigenvectors of ranks
// [k_lo, k_hi) for the keep form, the others for the removal form.
__global__ __launch_bounds__(1024) void rank_basis(const double* __restrict__ lam,
                                                   const double* __restrict__ v, int T, int k_lo,
                                                   int k_hi, int keep, float* __restrict__ sv,
                                                   float* __restrict__ Bm, int nb) {
  __shared__ int rank_of[kMaxT];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < T; i += nt) {
    const double li = lam[i];
    int rk = 0;
    for (int j = 0; j < T; ++j) {
      const double lj = lam[j];
      rk += (lj > li) || (lj == li && j < i);
    }
    rank_of[rk] = i;
    sv[rk] = (float)sqrt(fmax(li, 0.0));
  }
  __syncthreads();
  for (int w = tid; w < T * nb; w += nt) {
    const int t = w / nb, j = w - t * nb;
    const int rk = keep ? k_lo + j : (j < k_lo ? j : k_hi + (j - k_lo));
    Bm[w] = (float)v[(size_t)t * T + rank_of[rk]];
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

// Workspace layout (bytes from the start), every part 256-byte aligned:
// G, V, A, Y (T x T f64 each), sc (5 T x T f64: the tridiagonal factors),
// Bm (T x 64 f32), d, e, tau, lam (T f64 each).
struct ClutterWs {
  size_t G, V, A, Y, sc, Bm, d, e, tau, lam, total;
};
constexpr ClutterWs ws_layout(int T) {
  const size_t tt = align256(sizeof(double) * (size_t)T * T), t8 = align256(sizeof(double) * (size_t)T);
  ClutterWs L{};
  size_t o = 0;
  L.G = o; o += tt;
  L.V = o; o += tt;
  L.A = o; o += tt;
  L.Y = o; o += tt;
  L.sc = o; o += 5 * tt;
  L.Bm = o; o += align256(sizeof(float) * (size_t)T * 64);
  L.d = o; o += t8;
  L.e = o; o += t8;
  L.tau = o; o += t8;
  L.lam = o; o += t8;
  L.total = o;
  return L;
}
constexpr size_t workspace_bytes(int T) { return ws_layout(T).total; }

// Workspace of the allocation-free entry point: room for ensembles of up to
// kStaticT frames (4.6 MiB), one copy per device, held until the process
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
  double* sc = reinterpret_cast<double*>(w + L.sc);
  float* Bm = reinterpret_cast<float*>(w + L.Bm);
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
  const int nbk = (T + GB - 1) / GB, npairs = nbk * (nbk + 1) / 2;
  const long long nsteps = (N + GB - 1) / GB;
  const long long nchunk = std::max(1LL, std::min(nsteps, (long long)(8 * cus) / npairs + 1));
  const long long csz = (nsteps + nchunk - 1) / nchunk * GB;
  const long long nch = (N + csz - 1) / csz;
  hipLaunchKernelGGL(gram_mfma, dim3((unsigned)npairs, (unsigned)nch), dim3(256), 0, st, x, T, N,
                     csz, nbk, G);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tri_reduce, dim3(1), dim3(1024), 0, st, G, T, A, d, e_, tau);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tri_bisect, dim3(T), dim3(64), 0, st, d, e_, T, lam);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tri_inverse, dim3((T + 63) / 64), dim3(64), 0, st, d, e_, lam, T, sc, Y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tri_orth, dim3(1), dim3(1024), 0, st, lam, T, Y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(tri_back, dim3(T), dim3(256), 0, st, A, tau, Y, T, V);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(rank_basis, dim3(1), dim3(1024), 0, st, lam, V, T, k_lo, k_hi, keep, sv, Bm, nb);
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
