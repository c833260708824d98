// Global solve of the trace system H uhat = b (eq 6.5 after the Dirichlet elimination).
// The paper leaves the solver open; this is preconditioned conjugate gradients with a
// block-Jacobi preconditioner (explicit inverse of each d2 x d2 diagonal block, via its
// Cholesky factor).  One iteration is five launches: H p with the workgroup partials of
// p.Ap, their sum, the x and r updates fused with z = Minv r and the partials of r.z, their
// sum, and p = z + beta p.  Reductions are two-stage with a fixed grid and a fixed combining
// order, so every run gives the same bits.  alpha and beta live on the device; the host
// reads the residual norm every check_every iterations, and accepts the iterate only when
// the recomputed residual ||b - H x|| (FP64) meets the tolerance (otherwise the recursive
// residual is replaced by the true one and the iteration restarts from the current x).
//
// precision = 1: H and the preconditioner are also kept in FP32 and the correction
// equation H d = r is solved by an inner FP32-storage PCG inside an FP64 iterative
// refinement x <- x + d, r = b - H x (FP64 matrix, FP64 residuals and inner products).
#include <cmath>
#include <vector>

#include "device_common.h"

namespace hdg {
namespace {

constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

// ---- block-Jacobi setup: Minv[f] = (H_ff)^{-1}
template <int D2, class T>
__global__ void k_bj_setup(const double* __restrict__ H, const int* __restrict__ diag, int nfc, T* __restrict__ Minv) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfc) return;
  double A[D2][D2], X[D2][D2];
  const double* blk = H + (size_t)diag[f] * D2 * D2;
  for (int i = 0; i < D2; ++i)
    for (int j = 0; j < D2; ++j) A[i][j] = blk[i * D2 + j];
  for (int j = 0; j < D2; ++j) {  // Cholesky, lower
    double s = A[j][j];
    for (int k = 0; k < j; ++k) s -= A[j][k] * A[j][k];
    A[j][j] = sqrt(s);
    for (int i = j + 1; i < D2; ++i) {
      double v = A[i][j];
      for (int k = 0; k < j; ++k) v -= A[i][k] * A[j][k];
      A[i][j] = v / A[j][j];
    }
  }
  for (int c = 0; c < D2; ++c) {  // columns of the inverse
    double y[D2];
    for (int r = 0; r < D2; ++r) {
      double s = r == c ? 1.0 : 0.0;
      for (int k = 0; k < r; ++k) s -= A[r][k] * y[k];
      y[r] = s / A[r][r];
    }
    for (int r = D2 - 1; r >= 0; --r) {
      double s = y[r];
      for (int k = r + 1; k < D2; ++k) s -= A[k][r] * y[k];
      y[r] = s / A[r][r];
    }
    for (int r = 0; r < D2; ++r) X[r][c] = y[r];
  }
  T* o = Minv + (size_t)f * D2 * D2;
  for (int i = 0; i < D2; ++i)
    for (int j = 0; j < D2; ++j) o[i * D2 + j] = (T)(0.5 * (X[i][j] + X[j][i]));
}

// The same for the blocks of degrees 5 and 6 (d2 = 21, 28), too large for one thread's
// registers: one workgroup of 64 threads per face, the block factored in LDS (right-looking,
// one row per thread), then one column of the inverse per thread.
template <int D2, class T>
__global__ void __launch_bounds__(64) k_bj_setup_wg(const double* __restrict__ H, const int* __restrict__ diag,
                                                   int nfc, T* __restrict__ Minv) {
  __shared__ double A[D2][D2 + 1];
  __shared__ double X[D2][D2 + 1];
  const int t = threadIdx.x;
  for (int f = blockIdx.x; f < nfc; f += gridDim.x) {
    const double* blk = H + (size_t)diag[f] * D2 * D2;
    for (int i = t; i < D2 * D2; i += 64) A[i / D2][i % D2] = blk[i];
    __syncthreads();
    for (int j = 0; j < D2; ++j) {  // Cholesky, lower: column j from the updated trailing block
      const double d = sqrt(A[j][j]);
      __syncthreads();
      if (t >= j && t < D2) A[t][j] = t == j ? d : A[t][j] / d;
      __syncthreads();
      if (t > j && t < D2)
        for (int k = j + 1; k <= t; ++k) A[t][k] -= A[t][j] * A[k][j];
      __syncthreads();
    }
    if (t < D2) {  // column t of the inverse, kept in LDS
#pragma unroll 1
      for (int r = 0; r < D2; ++r) {
        double v = r == t ? 1.0 : 0.0;
#pragma unroll 4
        for (int k = 0; k < r; ++k) v -= A[r][k] * X[k][t];
        X[r][t] = v / A[r][r];
      }
#pragma unroll 1
      for (int r = D2 - 1; r >= 0; --r) {
        double v = X[r][t];
#pragma unroll 4
        for (int k = r + 1; k < D2; ++k) v -= A[k][r] * X[k][t];
        X[r][t] = v / A[r][r];
      }
    }
    __syncthreads();
    T* o = Minv + (size_t)f * D2 * D2;
    for (int i = t; i < D2 * D2; i += 64) {
      const int r = i / D2, c = i % D2;
      o[i] = (T)(0.5 * (X[r][c] + X[c][r]));
    }
    __syncthreads();
  }
}

// Minv[f] = (H_ff)^{-1} for every face, the form that suits the block size.
template <int D2, class T>
void launch_bj_setup(const double* H, const int* diag, int nfc, T* Minv, hipStream_t s) {
  if constexpr (D2 > 15)
    k_bj_setup_wg<D2, T><<<std::max(1, std::min(nfc, 8192)), 64, 0, s>>>(H, diag, nfc, Minv);
  else
    k_bj_setup<D2, T><<<(nfc + 63) / 64, 64, 0, s>>>(H, diag, nfc, Minv);
}

template <class T>
__global__ void k_convert(const double* __restrict__ a, T* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (T)a[i];
}

// Row entry c of block row f of H x, the blocks summed in storage order.
template <int D2, class TM, class TV>
__device__ __forceinline__ double row_dot(const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                                          const TM* __restrict__ H, const TV* __restrict__ x, int f, int c) {
  double s = 0;
  for (int p = row_ptr[f]; p < row_ptr[f + 1]; ++p) {
    const TM* blk = H + ((size_t)p * D2 + c) * D2;
    const TV* xv = x + (size_t)col_idx[p] * D2;
#pragma unroll
    for (int j = 0; j < D2; ++j) s += (double)blk[j] * (double)xv[j];
  }
  return s;
}

// ---- y = H x, one thread per row entry
template <int D2, class TM, class TV>
__global__ void k_spmv(const int* __restrict__ row_ptr, const int* __restrict__ col_idx, const TM* __restrict__ H,
                       const TV* __restrict__ x, TV* __restrict__ y, int nfc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfc * D2) return;
  y[i] = (TV)row_dot<D2>(row_ptr, col_idx, H, x, i / D2, i % D2);
}

// r = b - H x
template <int D2>
__global__ void k_residual(const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                           const double* __restrict__ H, const double* __restrict__ x, const double* __restrict__ b,
                           double* __restrict__ r, int nfc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfc * D2) return;
  r[i] = b[i] - row_dot<D2>(row_ptr, col_idx, H, x, i / D2, i % D2);
}

// ---- deterministic dot products: partial sums per block, fixed grid; final in one block
template <class TA, class TB>
__global__ void k_dot_partial(const TA* __restrict__ a, const TB* __restrict__ b, size_t n, double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double s = 0;
  for (size_t i = blockIdx.x * (size_t)kRedThreads + threadIdx.x; i < n; i += (size_t)kRedBlocks * kRedThreads)
    s += (double)a[i] * (double)b[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kRedThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_dot_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  double s = 0;
  for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kRedThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// z = Minv r (one thread per row entry)
template <int D2, class TM, class TV>
__global__ void k_precond(const TM* __restrict__ Minv, const TV* __restrict__ r, TV* __restrict__ z, int nfc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfc * D2) return;
  const int f = i / D2, c = i % D2;
  const TM* m = Minv + ((size_t)f * D2 + c) * D2;
  const TV* rv = r + (size_t)f * D2;
  double s = 0;
#pragma unroll
  for (int j = 0; j < D2; ++j) s += (double)m[j] * (double)rv[j];
  z[i] = (TV)s;
}

// Learned factor M^{-1} = L^{-T} G^T G L^{-1}, G = B (I + N) (N strictly block-lower, FP32,
// stored at the positions of the lower blocks of H with each transpose at the mirrored
// upper position; B the per-face block scaling; Linv the FP32 inverse Cholesky factors of
// the diagonal blocks).  Two sweeps, FP64 accumulation:
//   s_i = B_i^T B_i (t_i + sum_{j < i} N_ij t_j),  t = L^{-1} r   (lower blocks)
//   z_j = L_j^{-T} (s_j + sum_{i > j} N_ij^T s_i)                  (upper blocks)
// One thread per (face, component), the faces of a workgroup contiguous (Lpre::FACES), so
// that the threads of a face read whole block rows and the workgroup exchanges a face's
// components through LDS.
template <int D2>
struct Lpre {
  static constexpr int FACES = 256 / D2;
  static constexpr int THREADS = FACES * D2;
};

// t = L^{-1} r
template <int D2, class TV>
__global__ void __launch_bounds__(Lpre<D2>::THREADS) k_lpre_scale(const float* __restrict__ Linv,
                                                                  const TV* __restrict__ r, TV* __restrict__ t,
                                                                  int nfc) {
  const int i = blockIdx.x * Lpre<D2>::FACES + threadIdx.x / D2, a = threadIdx.x % D2;
  if (i >= nfc) return;
  const float* La = Linv + ((size_t)i * D2 + a) * D2;
  const TV* ri = r + (size_t)i * D2;
  double acc = 0.0;
#pragma unroll
  for (int b = 0; b < D2; ++b)
    if (b <= a) acc += (double)La[b] * (double)ri[b];
  t[(size_t)i * D2 + a] = (TV)acc;
}

// s_i = t_i + sum_{j < i} N_ij t_j: the lower blocks of row i are the entries before the
// diagonal (columns ascend).  With a block scaling (Bp not NULL) the kernel stores
// B_i^T B_i s_i instead: B_i lower triangular, B_i[a][a] = exp(Bp_i[a]),
// B_i[a][b] = Bp_i[D2 + a (a - 1) / 2 + b] (b < a); a face's components meet in LDS.
template <int D2, class TV>
__global__ void __launch_bounds__(Lpre<D2>::THREADS) k_lpre_lower(const int* __restrict__ row_ptr,
                                                                  const int* __restrict__ diag,
                                                                  const int* __restrict__ col,
                                                                  const float* __restrict__ N,
                                                                  const float* __restrict__ Bp,
                                                                  const TV* __restrict__ t, TV* __restrict__ s,
                                                                  int nfc) {
  constexpr int FB = D2 * (D2 + 1) / 2;
  __shared__ double sv[Lpre<D2>::THREADS];
  const int lf = threadIdx.x / D2, a = threadIdx.x % D2;
  const int i = blockIdx.x * Lpre<D2>::FACES + lf;
  double acc = 0.0;
  if (i < nfc) {
    const int e0 = row_ptr[i], e1 = diag[i];
    acc = (double)t[(size_t)i * D2 + a];
#pragma unroll 3
    for (int e = e0; e < e1; ++e) {
      const TV* tj = t + (size_t)col[e] * D2;
      const float* Na = N + ((size_t)e * D2 + a) * D2;
#pragma unroll
      for (int b = 0; b < D2; ++b) acc += (double)Na[b] * (double)tj[b];
    }
  }
  if (Bp) {  // uniform over the launch
    const float* bp = Bp + (size_t)(i < nfc ? i : 0) * FB;
    sv[threadIdx.x] = acc;
    __syncthreads();
    double v = exp((double)bp[a]) * sv[lf * D2 + a];  // v = B_i s_i
    for (int b = 0; b < a; ++b) v += (double)bp[D2 + a * (a - 1) / 2 + b] * sv[lf * D2 + b];
    __syncthreads();
    sv[threadIdx.x] = v;
    __syncthreads();
    acc = exp((double)bp[a]) * sv[lf * D2 + a];  // B_i^T v
    for (int c = a + 1; c < D2; ++c) acc += (double)bp[D2 + c * (c - 1) / 2 + a] * sv[lf * D2 + c];
  }
  if (i < nfc) s[(size_t)i * D2 + a] = (TV)acc;
}

// z_j = L_j^{-T} (s_j + sum_{i > j} N_ij^T s_i): the upper blocks of row j hold N_ij^T
// (hdg_gnn_forward writes each lower block's transpose at its mirrored position), so the
// sweep reads block rows contiguously, as the lower one does
template <int D2, class TV>
__global__ void __launch_bounds__(Lpre<D2>::THREADS) k_lpre_upper(const int* __restrict__ row_ptr,
                                                                  const int* __restrict__ diag,
                                                                  const int* __restrict__ col,
                                                                  const float* __restrict__ N,
                                                                  const float* __restrict__ Linv,
                                                                  const TV* __restrict__ s, TV* __restrict__ z,
                                                                  int nfc) {
  __shared__ double ys[Lpre<D2>::THREADS];
  const int lf = threadIdx.x / D2, a = threadIdx.x % D2;
  const int j = blockIdx.x * Lpre<D2>::FACES + lf;
  double y = 0.0;
  if (j < nfc) {
    y = (double)s[(size_t)j * D2 + a];
    const int e0 = diag[j] + 1, e1 = row_ptr[j + 1];
#pragma unroll 3
    for (int e = e0; e < e1; ++e) {
      const float* Nr = N + ((size_t)e * D2 + a) * D2;  // row a of N_ij^T
      const TV* si = s + (size_t)col[e] * D2;
#pragma unroll
      for (int b = 0; b < D2; ++b) y += (double)Nr[b] * (double)si[b];
    }
  }
  ys[threadIdx.x] = y;
  __syncthreads();
  if (j >= nfc) return;
  const float* Lj = Linv + (size_t)j * D2 * D2;
  double v = 0.0;
#pragma unroll
  for (int b = 0; b < D2; ++b)
    if (b >= a) v += (double)Lj[b * D2 + a] * ys[lf * D2 + b];
  z[(size_t)j * D2 + a] = (TV)v;
}

// ---- fused PCG iteration (block-Jacobi).  The scalars live on the device: scal[1] = p.Ap,
// and rz alternates between scal[0] and scal[2] (slot `old` holds r.z of the previous
// iteration, the other slot receives the new one), so no kernel has to shift them.
// Every reduction is per workgroup into part[], then k_sum_parts in a fixed order.

// Coalesced form for even block sizes (d2 = 6, 10): each row entry of a face is shared by
// d2/2 consecutive lanes, lane q taking columns 2q, 2q+1 of every block of the row, so that
// the d2 * d2/2 lanes of a face read each d2 x d2 block as one contiguous segment (one
// 16-byte load per lane in FP64) and the matching x pairs.  The faces of a workgroup are
// whole (FACES per workgroup); the partial sums of a row entry meet in LDS and are added in
// lane order.  With PAP, part[wg] = the workgroup's share of p.Ap.
template <int D2>
struct SpmvC {
  static_assert(D2 % 2 == 0 && D2 * D2 / 2 <= 256, "pairs of columns, a face's lanes in one workgroup");
  static constexpr int LPR = D2 / 2, LPF = D2 * LPR, FACES = 256 / LPF, THREADS = FACES * LPF;
};

template <class T>
struct Pair;
template <>
struct Pair<double> {
  using type = double2;
};
template <>
struct Pair<float> {
  using type = float2;
};

template <int D2, class TM, class TV, bool PAP>
__global__ void __launch_bounds__(256) k_spmv_c(const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                                                const TM* __restrict__ H, const TV* __restrict__ x,
                                                TV* __restrict__ y, int nfc, double* __restrict__ part) {
  using C = SpmvC<D2>;
  using PM = typename Pair<TM>::type;
  using PV = typename Pair<TV>::type;
  __shared__ double sh[256];
  const int t = threadIdx.x;
  const int lf = t / C::LPF, w = t % C::LPF, r = w / C::LPR, q = w % C::LPR;
  const int ngroups = (nfc + C::FACES - 1) / C::FACES;
  double contrib = 0;
  for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {  // uniform over the workgroup
    const int f = g * C::FACES + lf;
    const bool on = t < C::THREADS && f < nfc;
    double s = 0;
    if (on) {
      const int p1 = row_ptr[f + 1];
      int p = row_ptr[f];
      for (; p + 1 < p1; p += 2) {  // two blocks in flight
        const int c0 = col_idx[p], c1 = col_idx[p + 1];
        const PM h0 = *reinterpret_cast<const PM*>(H + ((size_t)p * D2 + r) * D2 + 2 * q);
        const PM h1 = *reinterpret_cast<const PM*>(H + ((size_t)(p + 1) * D2 + r) * D2 + 2 * q);
        const PV x0 = *reinterpret_cast<const PV*>(x + (size_t)c0 * D2 + 2 * q);
        const PV x1 = *reinterpret_cast<const PV*>(x + (size_t)c1 * D2 + 2 * q);
        s += (double)h0.x * (double)x0.x;
        s += (double)h0.y * (double)x0.y;
        s += (double)h1.x * (double)x1.x;
        s += (double)h1.y * (double)x1.y;
      }
      if (p < p1) {
        const PM h = *reinterpret_cast<const PM*>(H + ((size_t)p * D2 + r) * D2 + 2 * q);
        const PV xv = *reinterpret_cast<const PV*>(x + (size_t)col_idx[p] * D2 + 2 * q);
        s += (double)h.x * (double)xv.x;
        s += (double)h.y * (double)xv.y;
      }
    }
    __syncthreads();
    sh[t] = s;
    __syncthreads();
    if (on && q == 0) {
      double v = sh[t];
#pragma unroll
      for (int k = 1; k < C::LPR; ++k) v += sh[t + k];
      const size_t i = (size_t)f * D2 + r;
      const TV yv = (TV)v;
      y[i] = yv;
      if (PAP) contrib += (double)yv * (double)x[i];
    }
  }
  if (PAP) {
    __syncthreads();
    sh[t] = contrib;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) sh[t] += sh[t + o];
      __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = sh[0];
  }
}

// Ap = H p (one thread per row entry, 256 per workgroup) and part[wg] = sum of p.Ap over the
// workgroup's rows
template <int D2, class TM, class TV>
__global__ void __launch_bounds__(256) k_spmv_pap(const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                                                  const TM* __restrict__ H, const TV* __restrict__ x,
                                                  TV* __restrict__ y, int nfc, double* __restrict__ part) {
  __shared__ double sh[256];
  double contrib = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nfc * D2; i += gridDim.x * 256) {
    const TV yv = (TV)row_dot<D2>(row_ptr, col_idx, H, x, i / D2, i % D2);
    y[i] = yv;
    contrib += (double)yv * (double)x[i];
  }
  sh[threadIdx.x] = contrib;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Ap = H p with part[wg] = the workgroup's share of p.Ap; returns the number of partials.
constexpr int kMaxParts = 2048;

// y = H x (FP64), the coalesced kernel where the block size allows it
template <int D2>
void launch_spmv(const hdg_mesh* mesh, const double* H, const double* x, double* y, hipStream_t s) {
  const int nfc = (int)mesh->nfc;
  if constexpr (D2 % 2 == 0 && D2 >= 6 && D2 * D2 / 2 <= 256) {
    const int groups = (nfc + SpmvC<D2>::FACES - 1) / SpmvC<D2>::FACES;
    k_spmv_c<D2, double, double, false><<<std::max(1, std::min(groups, kMaxParts)), 256, 0, s>>>(
        mesh->d_row_ptr, mesh->d_col_idx, H, x, y, nfc, nullptr);
  } else {
    k_spmv<D2, double, double><<<(unsigned)((nfc * D2 + 255) / 256), 256, 0, s>>>(mesh->d_row_ptr, mesh->d_col_idx,
                                                                                   H, x, y, nfc);
  }
}

template <int D2, class TM, class TV>
int launch_spmv_pap(const hdg_mesh* mesh, const TM* H, const TV* x, TV* y, double* part, hipStream_t s) {
  const int nfc = (int)mesh->nfc;
  if constexpr (D2 % 2 == 0 && D2 >= 6 && D2 * D2 / 2 <= 256 && sizeof(TM) == 8) {  // 16-byte pairs (FP64 H)
    const int groups = (nfc + SpmvC<D2>::FACES - 1) / SpmvC<D2>::FACES;
    const int g = std::max(1, std::min(groups, kMaxParts));
    k_spmv_c<D2, TM, TV, true><<<g, 256, 0, s>>>(mesh->d_row_ptr, mesh->d_col_idx, H, x, y, nfc, part);
    return g;
  } else {
    const int g = std::max(1, std::min((nfc * D2 + 255) / 256, kMaxParts));
    k_spmv_pap<D2, TM, TV><<<g, 256, 0, s>>>(mesh->d_row_ptr, mesh->d_col_idx, H, x, y, nfc, part);
    return g;
  }
}

// out = sum of part[0..count) in a fixed order (one workgroup of kSumThreads threads, four
// independent accumulators per thread so that its loads overlap)
constexpr int kSumThreads = 1024;

__global__ void __launch_bounds__(kSumThreads) k_sum_parts(const double* __restrict__ part, int count,
                                                           double* __restrict__ out) {
  __shared__ double sh[kSumThreads];
  double a[4] = {0, 0, 0, 0};
  int i = threadIdx.x;
  for (; i + 3 * kSumThreads < count; i += 4 * kSumThreads) {
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] += part[i + q * kSumThreads];
  }
  for (int q = 0; i < count; i += kSumThreads, ++q) a[q] += part[i];
  sh[threadIdx.x] = (a[0] + a[1]) + (a[2] + a[3]);
  __syncthreads();
  for (int o = kSumThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// x += alpha p, r -= alpha Ap (alpha = scal[old] / scal[1]), z = Minv r with a face's
// components exchanged in LDS, part[wg] = sum of r.z over the workgroup's faces
template <int D2, class TM, class TV>
__global__ void __launch_bounds__(Lpre<D2>::THREADS) k_xr_precond_rz(TV* __restrict__ x, TV* __restrict__ r,
                                                                     const TV* __restrict__ p,
                                                                     const TV* __restrict__ Ap,
                                                                     const TM* __restrict__ Minv, TV* __restrict__ z,
                                                                     const double* __restrict__ scal, int old, int nfc,
                                                                     double* __restrict__ part) {
  __shared__ double rs[Lpre<D2>::THREADS];
  __shared__ double sh[256];
  const int lf = threadIdx.x / D2, c = threadIdx.x % D2;
  const double alpha = scal[old] / scal[1];
  const int ngroups = (nfc + Lpre<D2>::FACES - 1) / Lpre<D2>::FACES;
  double contrib = 0.0;
  for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {  // uniform over the workgroup
    const int f = g * Lpre<D2>::FACES + lf;
    const size_t i = (size_t)f * D2 + c;
    double rn = 0.0;
    if (f < nfc) {
      x[i] = (TV)((double)x[i] + alpha * (double)p[i]);
      const TV rv = (TV)((double)r[i] - alpha * (double)Ap[i]);
      r[i] = rv;
      rn = (double)rv;
    }
    __syncthreads();
    rs[threadIdx.x] = rn;
    __syncthreads();
    if (f < nfc) {
      const TM* m = Minv + ((size_t)f * D2 + c) * D2;
      double acc = 0;
#pragma unroll
      for (int j = 0; j < D2; ++j) acc += (double)m[j] * rs[lf * D2 + j];
      const TV zv = (TV)acc;
      z[i] = zv;
      contrib += rn * (double)zv;
    }
  }
  sh[threadIdx.x] = contrib;
  if (threadIdx.x < 256 - Lpre<D2>::THREADS) sh[Lpre<D2>::THREADS + threadIdx.x] = 0.0;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// The learned form's first stage fused with the x and r updates: x += alpha p,
// r -= alpha Ap, t = L^{-1} r per face (L^{-1} lower triangular, FP32), a face's
// components exchanged in LDS
template <int D2, class TV>
__global__ void __launch_bounds__(Lpre<D2>::THREADS) k_xr_lscale(TV* __restrict__ x, TV* __restrict__ r,
                                                                 const TV* __restrict__ p, const TV* __restrict__ Ap,
                                                                 const float* __restrict__ Linv, TV* __restrict__ t,
                                                                 const double* __restrict__ scal, int old, int nfc) {
  __shared__ double rs[Lpre<D2>::THREADS];
  const int lf = threadIdx.x / D2, c = threadIdx.x % D2;
  const double alpha = scal[old] / scal[1];
  const int ngroups = (nfc + Lpre<D2>::FACES - 1) / Lpre<D2>::FACES;
  for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {  // uniform over the workgroup
    const int f = g * Lpre<D2>::FACES + lf;
    const size_t i = (size_t)f * D2 + c;
    double rn = 0.0;
    if (f < nfc) {
      x[i] = (TV)((double)x[i] + alpha * (double)p[i]);
      const TV rv = (TV)((double)r[i] - alpha * (double)Ap[i]);
      r[i] = rv;
      rn = (double)rv;
    }
    __syncthreads();
    rs[threadIdx.x] = rn;
    __syncthreads();
    if (f < nfc) {
      const float* La = Linv + ((size_t)f * D2 + c) * D2;
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < D2; ++b)
        if (b <= c) acc += (double)La[b] * rs[lf * D2 + b];
      t[i] = (TV)acc;
    }
  }
}

// p = z + beta p with beta = scal[nw] / scal[old]
template <class TV>
__global__ void k_update_p_slot(TV* __restrict__ p, const TV* __restrict__ z, const double* __restrict__ scal, int old,
                                int nw, size_t n) {
  const double beta = scal[nw] / scal[old];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = (TV)((double)z[i] + beta * (double)p[i]);
}

template <class TV>
__global__ void k_copy(const TV* __restrict__ a, TV* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = a[i];
}

template <class TA, class TB>
__global__ void k_axpy_cast(const TA* __restrict__ a, TB* __restrict__ b, size_t n) {  // b += a
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (TB)((double)b[i] + (double)a[i]);
}

template <class TV>
__global__ void k_fill(TV* __restrict__ a, size_t n, double v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) a[i] = (TV)v;
}

template <class TA, class TB>
__global__ void k_scale_cast(const TA* __restrict__ a, TB* __restrict__ b, size_t n, const double* __restrict__ nrm) {
  const double s = 1.0 / sqrt(*nrm);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (TB)((double)a[i] * s);
}

template <class TA, class TB>
__global__ void k_axpy_scaled(const TA* __restrict__ a, TB* __restrict__ b, size_t n, const double* __restrict__ nrm) {
  const double s = sqrt(*nrm);  // b += s * a
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (TB)((double)b[i] + s * (double)a[i]);
}

struct Carve {
  char* p;
  size_t left;
  bool ok = true;
  template <class T>
  T* take(size_t n) {
    size_t bytes = (n * sizeof(T) + 255) & ~size_t(255);
    if (bytes > left) { ok = false; return nullptr; }
    T* r = reinterpret_cast<T*>(p);
    p += bytes;
    left -= bytes;
    return r;
  }
};

// Partial sums: one per workgroup of the fused PCG kernels (at most kMaxParts), and the
// kRedBlocks of the plain dot products.
size_t part_count(size_t) { return std::max<size_t>(kRedBlocks, kMaxParts); }

size_t ws_size(const hdg_mesh* mesh, int d2, int precision) {
  const size_t n = (size_t)mesh->nfc * d2;
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  for (int i = 0; i < 5; ++i) add(n * sizeof(double));  // r z p Ap, and the learned factor's sweep
  add((size_t)mesh->nfc * d2 * d2 * sizeof(double));    // Minv
  add(part_count(n) * sizeof(double));
  add(8 * sizeof(double));
  if (precision == 1) {
    for (int i = 0; i < 6; ++i) add(n * sizeof(float));  // d r z p Ap sweep (inner)
    add((size_t)mesh->nnzb * d2 * d2 * sizeof(float));   // H in FP32
    add((size_t)mesh->nfc * d2 * d2 * sizeof(float));    // Minv in FP32
  }
  return b;
}

template <int D2>
struct Solver {
  const hdg_mesh* mesh;
  hipStream_t s;
  size_t n;
  unsigned gv, gr;
  double* part;
  double* scal;

  template <class TA, class TB>
  void dot(const TA* a, const TB* b, double* out) {
    k_dot_partial<<<kRedBlocks, kRedThreads, 0, s>>>(a, b, n, part);
    k_dot_final<<<1, kRedThreads, 0, s>>>(part, out);
  }
  double read(const double* d) {
    double h = 0;
    (void)hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    return h;
  }
};

template <int D2>
hdg_status run_solve(const hdg_mesh* mesh, const double* H, const double* b, double* x, const hdg_solve_opts* o,
                     hdg_solve_info* info, void* ws, size_t ws_bytes, hipStream_t s) {
  const size_t n = (size_t)mesh->nfc * D2;
  Carve cv{(char*)ws, ws_bytes};
  double* r = cv.take<double>(n);
  double* z = cv.take<double>(n);
  double* p = cv.take<double>(n);
  double* Ap = cv.take<double>(n);
  double* sw = cv.take<double>(n);
  double* Minv = cv.take<double>((size_t)mesh->nfc * D2 * D2);
  double* part = cv.take<double>(part_count(n));
  double* scal = cv.take<double>(8);
  float *d32 = nullptr, *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *Ap32 = nullptr, *H32 = nullptr,
        *Minv32 = nullptr, *sw32 = nullptr;
  if (o->precision == 1) {
    sw32 = cv.take<float>(n);
    d32 = cv.take<float>(n);
    r32 = cv.take<float>(n);
    z32 = cv.take<float>(n);
    p32 = cv.take<float>(n);
    Ap32 = cv.take<float>(n);
    H32 = cv.take<float>((size_t)mesh->nnzb * D2 * D2);
    Minv32 = cv.take<float>((size_t)mesh->nfc * D2 * D2);
  }
  if (!cv.ok) return set_error(HDG_ERR_WORKSPACE, "hdg_solve: workspace too small");
  const unsigned T = 256;
  const unsigned gv = (unsigned)std::min<size_t>((n + T - 1) / T, 8192);
  const unsigned gr = (unsigned)((n + T - 1) / T);
  Solver<D2> S{mesh, s, n, gv, gr, part, scal};
  const int nfc = (int)mesh->nfc;
  constexpr bool kLearn = D2 <= 15;  // the learned factor exists for degrees 0..4
  const bool learned = kLearn && o->precond == 1;
  const unsigned gf = (unsigned)((nfc + Lpre<D2>::FACES - 1) / Lpre<D2>::FACES);
  constexpr unsigned TL = Lpre<D2>::THREADS;
  auto pre64 = [&](const double* rr_, double* zz_) {
    if constexpr (kLearn) {
      if (learned) {  // t -> zz_, s -> sw, then z -> zz_
        k_lpre_scale<D2, double><<<gf, TL, 0, s>>>(o->d_pre_Linv, rr_, zz_, nfc);
        k_lpre_lower<D2, double><<<gf, TL, 0, s>>>(mesh->d_row_ptr, mesh->d_diag, mesh->d_col_idx, o->d_pre_N,
                                                   o->d_pre_B, zz_, sw, nfc);
        k_lpre_upper<D2, double><<<gf, TL, 0, s>>>(mesh->d_row_ptr, mesh->d_diag, mesh->d_col_idx, o->d_pre_N,
                                                   o->d_pre_Linv, sw, zz_, nfc);
        return;
      }
    }
    k_precond<D2, double, double><<<gr, T, 0, s>>>(Minv, rr_, zz_, nfc);
  };
  auto pre32 = [&](const float* rr_, float* zz_) {
    if constexpr (kLearn) {
      if (learned) {
        k_lpre_scale<D2, float><<<gf, TL, 0, s>>>(o->d_pre_Linv, rr_, zz_, nfc);
        k_lpre_lower<D2, float><<<gf, TL, 0, s>>>(mesh->d_row_ptr, mesh->d_diag, mesh->d_col_idx, o->d_pre_N,
                                                  o->d_pre_B, zz_, sw32, nfc);
        k_lpre_upper<D2, float><<<gf, TL, 0, s>>>(mesh->d_row_ptr, mesh->d_diag, mesh->d_col_idx, o->d_pre_N,
                                                  o->d_pre_Linv, sw32, zz_, nfc);
        return;
      }
    }
    k_precond<D2, float, float><<<gr, T, 0, s>>>(Minv32, rr_, zz_, nfc);
  };
  launch_bj_setup<D2, double>(H, mesh->d_diag, nfc, Minv, s);
  // ||b||
  S.dot(b, b, scal + 4);
  const double bb = S.read(scal + 4);
  HDG_CHECK_LAUNCH("hdg_solve setup");
  info->iterations = 0;
  info->outer = 0;
  info->rel_residual = 0;
  if (bb == 0) {
    k_fill<double><<<gv, T, 0, s>>>(x, n, 0.0);
    return HDG_OK;
  }
  const double tol2 = o->rtol * o->rtol * bb;
  const int every = std::max(1, o->check_every);
  const unsigned gfp = std::max(1u, std::min(gf, (unsigned)kMaxParts));  // k_xr_precond_rz grid
  // rz of the previous iteration is in slot old(it), the new one goes to the other slot
  auto old_slot = [](int it) { return (it & 1) ? 2 : 0; };
  if (o->precision == 0) {
    k_residual<D2><<<gr, T, 0, s>>>(mesh->d_row_ptr, mesh->d_col_idx, H, x, b, r, nfc);
    pre64(r, z);
    k_copy<double><<<gv, T, 0, s>>>(z, p, n);
    S.dot(r, z, scal + 0);
    int it = 0;
    for (;;) {
      if (it % every == 0 || it >= o->max_iter) {
        S.dot(r, r, scal + 3);
        double rr = S.read(scal + 3);
        HDG_CHECK_LAUNCH("hdg_solve");
        if (!std::isfinite(rr)) {
          info->iterations = it;
          info->rel_residual = std::nan("");
          return set_error(HDG_ERR_NOT_CONVERGED, "hdg_solve: breakdown (non-finite residual)");
        }
        if (rr <= tol2 || it >= o->max_iter) {
          // verify with the recomputed residual
          k_residual<D2><<<gr, T, 0, s>>>(mesh->d_row_ptr, mesh->d_col_idx, H, x, b, r, nfc);
          S.dot(r, r, scal + 3);
          double tr = S.read(scal + 3);
          info->iterations = it;
          info->rel_residual = std::sqrt(tr / bb);
          if (tr <= tol2) return HDG_OK;
          if (it >= o->max_iter)
            return set_error(HDG_ERR_NOT_CONVERGED, "hdg_solve: iteration limit reached");
          // residual replacement and restart
          pre64(r, z);
          k_copy<double><<<gv, T, 0, s>>>(z, p, n);
          S.dot(r, z, scal + old_slot(it));
        }
      }
      const int od = old_slot(it), nw = 2 - od;
      const int np1 = launch_spmv_pap<D2>(mesh, H, p, Ap, part, s);
      k_sum_parts<<<1, kSumThreads, 0, s>>>(part, np1, scal + 1);
      if (kLearn && learned) {  // t -> z, s -> sw, then z
        if constexpr (kLearn) {
          k_xr_lscale<D2, double><<<gfp, TL, 0, s>>>(x, r, p, Ap, o->d_pre_Linv, z, scal, od, nfc);
          k_lpre_lower<D2, double><<<gf, TL, 0, s>>>(mesh->d_row_ptr, mesh->d_diag, mesh->d_col_idx, o->d_pre_N,
                                                     o->d_pre_B, z, sw, nfc);
          k_lpre_upper<D2, double><<<gf, TL, 0, s>>>(mesh->d_row_ptr, mesh->d_diag, mesh->d_col_idx, o->d_pre_N,
                                                     o->d_pre_Linv, sw, z, nfc);
          S.dot(r, z, scal + nw);
        }
      } else {
        k_xr_precond_rz<D2, double, double><<<gfp, TL, 0, s>>>(x, r, p, Ap, Minv, z, scal, od, nfc, part);
        k_sum_parts<<<1, kSumThreads, 0, s>>>(part, (int)gfp, scal + nw);
      }
      k_update_p_slot<double><<<gv, T, 0, s>>>(p, z, scal, od, nw, n);
      ++it;
    }
  }
  // ---- precision 1: FP64 refinement around an FP32-storage PCG
  const size_t nh = (size_t)mesh->nnzb * D2 * D2;
  k_convert<float><<<8192, T, 0, s>>>(H, H32, nh);
  launch_bj_setup<D2, float>(H, mesh->d_diag, nfc, Minv32, s);
  int total = 0;
  const double inner_rtol = 1e-4;
  for (int outer = 0; outer < 60; ++outer) {
    k_residual<D2><<<gr, T, 0, s>>>(mesh->d_row_ptr, mesh->d_col_idx, H, x, b, r, nfc);
    S.dot(r, r, scal + 5);
    const double rr = S.read(scal + 5);
    HDG_CHECK_LAUNCH("hdg_solve refinement");
    info->outer = outer;
    info->iterations = total;
    info->rel_residual = std::sqrt(rr / bb);
    if (!std::isfinite(rr)) {
      info->rel_residual = std::nan("");
      return set_error(HDG_ERR_NOT_CONVERGED, "hdg_solve: breakdown in refinement");
    }
    if (rr <= tol2) return HDG_OK;
    if (total >= o->max_iter) return set_error(HDG_ERR_NOT_CONVERGED, "hdg_solve: iteration limit reached");
    // inner: H d = r / ||r|| in FP32 storage, d = 0
    k_scale_cast<double, float><<<gv, T, 0, s>>>(r, r32, n, scal + 5);
    k_fill<float><<<gv, T, 0, s>>>(d32, n, 0.0);
    pre32(r32, z32);
    k_copy<float><<<gv, T, 0, s>>>(z32, p32, n);
    S.dot(r32, z32, scal + 0);
    const double in_tol2 = inner_rtol * inner_rtol;  // relative to ||r32|| = 1
    for (int it = 0;; ++it) {
      if (it % every == 0) {
        S.dot(r32, r32, scal + 3);
        double r2 = S.read(scal + 3);
        if (!(r2 > in_tol2) || total >= o->max_iter) break;
      }
      const int od = old_slot(it), nw = 2 - od;
      const int np1 = launch_spmv_pap<D2>(mesh, H32, p32, Ap32, part, s);
      k_sum_parts<<<1, kSumThreads, 0, s>>>(part, np1, scal + 1);
      if (kLearn && learned) {
        if constexpr (kLearn) {
          k_xr_lscale<D2, float><<<gfp, TL, 0, s>>>(d32, r32, p32, Ap32, o->d_pre_Linv, z32, scal, od, nfc);
          k_lpre_lower<D2, float><<<gf, TL, 0, s>>>(mesh->d_row_ptr, mesh->d_diag, mesh->d_col_idx, o->d_pre_N,
                                                    o->d_pre_B, z32, sw32, nfc);
          k_lpre_upper<D2, float><<<gf, TL, 0, s>>>(mesh->d_row_ptr, mesh->d_diag, mesh->d_col_idx, o->d_pre_N,
                                                    o->d_pre_Linv, sw32, z32, nfc);
          S.dot(r32, z32, scal + nw);
        }
      } else {
        k_xr_precond_rz<D2, float, float><<<gfp, TL, 0, s>>>(d32, r32, p32, Ap32, Minv32, z32, scal, od, nfc, part);
        k_sum_parts<<<1, kSumThreads, 0, s>>>(part, (int)gfp, scal + nw);
      }
      k_update_p_slot<float><<<gv, T, 0, s>>>(p32, z32, scal, od, nw, n);
      ++total;
    }
    k_axpy_scaled<float, double><<<gv, T, 0, s>>>(d32, x, n, scal + 5);
  }
  return set_error(HDG_ERR_NOT_CONVERGED, "hdg_solve: refinement did not converge");
}

}  // namespace

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who);

}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_solve_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, int precision,
                                               size_t* ws_bytes) {
  if (!disc || !mesh || !ws_bytes) return set_error(HDG_ERR_INVALID_ARG, "hdg_solve_workspace_size: NULL argument");
  if (precision != 0 && precision != 1) return set_error(HDG_ERR_INVALID_ARG, "hdg_solve_workspace_size: precision");
  *ws_bytes = ws_size(mesh, disc->host.d2, precision);
  return HDG_OK;
}

extern "C" hdg_status hdg_solve(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_H, const double* d_b,
                                double* d_uhat, const hdg_solve_opts* opts, hdg_solve_info* info, void* d_ws,
                                size_t ws_bytes, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_solve");
  if (st) return st;
  if (!d_H || !d_b || !d_uhat || !opts || !info || !mesh->d_row_ptr || !mesh->d_col_idx)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_solve: NULL argument");
  if (!(opts->rtol > 0) || opts->max_iter < 0 || (opts->precision != 0 && opts->precision != 1) ||
      (opts->precond != 0 && opts->precond != 1))
    return set_error(HDG_ERR_INVALID_ARG, "hdg_solve: bad options");
  if (opts->precond == 1 && (!opts->d_pre_N || !opts->d_pre_Linv))
    return set_error(HDG_ERR_INVALID_ARG, "hdg_solve: the learned preconditioner needs N and Linv");
  if (opts->precond == 1 && disc->host.k > kMaxBatchDegree)
    return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_solve: the learned preconditioner exists for degrees 0..4");
  if (!d_ws || ws_bytes < ws_size(mesh, disc->host.d2, opts->precision))
    return set_error(HDG_ERR_WORKSPACE, "hdg_solve: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  auto run = [&](const hdg_solve_opts* o, hdg_solve_info* inf) -> hdg_status {
    switch (disc->host.k) {
      case 0: return run_solve<dim2(0)>(mesh, d_H, d_b, d_uhat, o, inf, d_ws, ws_bytes, s);
      case 1: return run_solve<dim2(1)>(mesh, d_H, d_b, d_uhat, o, inf, d_ws, ws_bytes, s);
      case 2: return run_solve<dim2(2)>(mesh, d_H, d_b, d_uhat, o, inf, d_ws, ws_bytes, s);
      case 3: return run_solve<dim2(3)>(mesh, d_H, d_b, d_uhat, o, inf, d_ws, ws_bytes, s);
      case 4: return run_solve<dim2(4)>(mesh, d_H, d_b, d_uhat, o, inf, d_ws, ws_bytes, s);
      case 5: return run_solve<dim2(5)>(mesh, d_H, d_b, d_uhat, o, inf, d_ws, ws_bytes, s);
      case 6: return run_solve<dim2(6)>(mesh, d_H, d_b, d_uhat, o, inf, d_ws, ws_bytes, s);
    }
    return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_solve: unsupported degree");
  };
  info->fell_back = 0;
  hdg_status st2 = run(opts, info);
  if (st2 != HDG_ERR_NOT_CONVERGED || opts->precond == 0) return st2;
  // fallback: block-Jacobi from the current iterate (or from zero after a breakdown)
  const int used = info->iterations;
  hdg_solve_opts bj = *opts;
  bj.precond = 0;
  if (!std::isfinite(info->rel_residual) || info->rel_residual > 1.0) {
    const size_t n = (size_t)mesh->nfc * disc->host.d2;
    k_fill<double><<<(unsigned)std::min<size_t>((n + 255) / 256, 8192), 256, 0, s>>>(d_uhat, n, 0.0);
    HDG_CHECK_LAUNCH("hdg_solve: fallback reset");
  }
  st2 = run(&bj, info);
  info->fell_back = 1;
  info->iterations += used;
  return st2;
}

namespace hdg {
namespace {
template <int D2>
void lpre_apply64(const hdg_mesh* mesh, const float* N, const float* Bp, const float* Linv, const double* r, double* z,
                  double* tmp, hipStream_t s) {
  const int nfc = (int)mesh->nfc;
  const unsigned gf = (unsigned)((nfc + Lpre<D2>::FACES - 1) / Lpre<D2>::FACES);
  constexpr unsigned TL = Lpre<D2>::THREADS;
  k_lpre_scale<D2, double><<<gf, TL, 0, s>>>(Linv, r, z, nfc);
  k_lpre_lower<D2, double><<<gf, TL, 0, s>>>(mesh->d_row_ptr, mesh->d_diag, mesh->d_col_idx, N, Bp, z, tmp, nfc);
  k_lpre_upper<D2, double><<<gf, TL, 0, s>>>(mesh->d_row_ptr, mesh->d_diag, mesh->d_col_idx, N, Linv, tmp, z, nfc);
}
}  // namespace
}  // namespace hdg

extern "C" hdg_status hdg_gnn_precond_apply(const hdg_disc* disc, const hdg_mesh* mesh, const float* d_N,
                                            const float* d_B, const float* d_Linv, const double* d_r,
                                            double* d_z, void* d_ws, size_t ws_bytes, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_gnn_precond_apply");
  if (st) return st;
  if (!d_N || !d_Linv || !d_r || !d_z || !mesh->d_row_ptr || !mesh->d_col_idx)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_precond_apply: NULL argument");
  if (d_r == d_z) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_precond_apply: r and z must not overlap");
  const size_t need = (size_t)mesh->nfc * disc->host.d2 * sizeof(double);
  if (!d_ws || ws_bytes < need) return set_error(HDG_ERR_WORKSPACE, "hdg_gnn_precond_apply: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  double* tmp = (double*)d_ws;
  switch (disc->host.k) {
    case 0: lpre_apply64<dim2(0)>(mesh, d_N, d_B, d_Linv, d_r, d_z, tmp, s); break;
    case 1: lpre_apply64<dim2(1)>(mesh, d_N, d_B, d_Linv, d_r, d_z, tmp, s); break;
    case 2: lpre_apply64<dim2(2)>(mesh, d_N, d_B, d_Linv, d_r, d_z, tmp, s); break;
    case 3: lpre_apply64<dim2(3)>(mesh, d_N, d_B, d_Linv, d_r, d_z, tmp, s); break;
    case 4: lpre_apply64<dim2(4)>(mesh, d_N, d_B, d_Linv, d_r, d_z, tmp, s); break;
    default: return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_gnn_precond_apply: unsupported degree");
  }
  HDG_CHECK_LAUNCH("hdg_gnn_precond_apply");
  return HDG_OK;
}

// ---------------------------------------------------------------------------------------
// GMRES for non-symmetric trace systems (the convection-diffusion HDG): restarted GMRES(m)
// with right block-Jacobi preconditioning (explicit inverses of the d2 x d2 diagonal blocks
// by Gauss-Jordan with partial pivoting), classical Gram-Schmidt with a second pass under
// severe cancellation, fixed-order reductions.  The small Hessenberg least-squares problem
// (Givens rotations) is solved on the host; the host reads one column of it per iteration.
namespace hdg {
namespace {

template <int D2>
__global__ void k_bj_setup_lu(const double* __restrict__ H, const int* __restrict__ diag, int nfc,
                              double* __restrict__ Minv) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfc) return;
  double A[D2][2 * D2];
  const double* blk = H + (size_t)diag[f] * D2 * D2;
  for (int i = 0; i < D2; ++i)
    for (int j = 0; j < D2; ++j) {
      A[i][j] = blk[i * D2 + j];
      A[i][D2 + j] = i == j ? 1.0 : 0.0;
    }
  for (int c = 0; c < D2; ++c) {
    int piv = c;
    for (int r = c + 1; r < D2; ++r)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    if (piv != c)
      for (int j = 0; j < 2 * D2; ++j) {
        const double t = A[c][j];
        A[c][j] = A[piv][j];
        A[piv][j] = t;
      }
    const double inv = 1.0 / A[c][c];
    for (int j = 0; j < 2 * D2; ++j) A[c][j] *= inv;
    for (int r = 0; r < D2; ++r)
      if (r != c) {
        const double m = A[r][c];
        for (int j = 0; j < 2 * D2; ++j) A[r][j] -= m * A[c][j];
      }
  }
  double* o = Minv + (size_t)f * D2 * D2;
  for (int i = 0; i < D2; ++i)
    for (int j = 0; j < D2; ++j) o[i * D2 + j] = A[i][D2 + j];
}

// part[b * nt + i] = partial (w, V_i) of block b for i < nv, and with self = 1 also
// part[b * nt + nv] = partial (w, w); nt = nv + self.  The products are taken eight at a
// time: one pass over the rows accumulates all eight in registers, and one tree reduction in
// LDS finishes the eight together.
constexpr int kMdotChunk = 8;
constexpr int kMdotBlocks = 2048;  // enough waves in flight to stream the basis from HBM

__global__ void __launch_bounds__(kRedThreads) k_mdot_partial(const double* __restrict__ V, size_t ldv, int nv,
                                                              int self, const double* __restrict__ w, size_t n,
                                                              double* __restrict__ part) {
  __shared__ double sh[kMdotChunk][kRedThreads];
  const int nt = nv + self;
  for (int i0 = 0; i0 < nt; i0 += kMdotChunk) {
    const int cnt = min(kMdotChunk, nt - i0);
    double acc[kMdotChunk];
#pragma unroll
    for (int q = 0; q < kMdotChunk; ++q) acc[q] = 0;
    for (size_t t = blockIdx.x * (size_t)kRedThreads + threadIdx.x; t < n; t += (size_t)kMdotBlocks * kRedThreads) {
      const double wt = w[t];
#pragma unroll
      for (int q = 0; q < kMdotChunk; ++q)
        if (q < cnt) acc[q] += wt * (i0 + q < nv ? V[(size_t)(i0 + q) * ldv + t] : wt);
    }
#pragma unroll
    for (int q = 0; q < kMdotChunk; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o)
#pragma unroll
        for (int q = 0; q < kMdotChunk; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + o];
      __syncthreads();
    }
    if ((int)threadIdx.x < cnt) part[(size_t)blockIdx.x * nt + i0 + threadIdx.x] = sh[threadIdx.x][0];
    __syncthreads();
  }
}

// out[i] (+)= sum over the blocks of part[b * nv + i], one workgroup per i
__global__ void k_mdot_final(const double* __restrict__ part, int nv, double* __restrict__ out, int accumulate) {
  __shared__ double sh[kRedThreads];
  const int i = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < kMdotBlocks; b += kRedThreads) s += part[(size_t)b * nv + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kRedThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = accumulate ? out[i] + sh[0] : sh[0];
}

// w -= sum_i h[i] V_i
__global__ void k_sub_combination(double* __restrict__ w, const double* __restrict__ V, size_t ldv, int nv,
                                  const double* __restrict__ h, size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    double s = w[t];
    for (int i = 0; i < nv; ++i) s -= h[i] * V[(size_t)i * ldv + t];
    w[t] = s;
  }
}

// y = sum_i c[i] V_i
__global__ void k_combination(double* __restrict__ y, const double* __restrict__ V, size_t ldv, int nv,
                              const double* __restrict__ c, size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    double s = 0;
    for (int i = 0; i < nv; ++i) s += c[i] * V[(size_t)i * ldv + t];
    y[t] = s;
  }
}

// v = w / sqrt(nrm2[0]) (or w / a for a given scalar when nrm2 == NULL)
__global__ void k_scale_into(double* __restrict__ v, const double* __restrict__ w, const double* __restrict__ nrm2,
                             double a, size_t n) {
  const double d = nrm2 ? sqrt(nrm2[0]) : a;
  const double inv = 1.0 / d;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
    v[t] = w[t] * inv;
}

__global__ void k_add_into(double* __restrict__ x, const double* __restrict__ z, size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
    x[t] += z[t];
}

constexpr int kMaxRestart = 64;

// Workspace, in doubles: the m + 1 basis vectors, w, z, r, the inverse diagonal blocks, the
// partial sums of the batched dots, and a small device array (both Gram-Schmidt passes'
// coefficients, the norm, y).
size_t gmres_ws_doubles(size_t n, int nfc, int d2, int m) {
  return (size_t)(m + 4) * n + (size_t)nfc * d2 * d2 + (size_t)kMdotBlocks * (m + 2) + 3 * (size_t)(m + 2) + 64;
}

template <int D2>
hdg_status run_gmres(const hdg_mesh* mesh, const double* H, const double* b, double* x, double rtol, int max_iter,
                     int m, hdg_solve_info* info, double* ws, hipStream_t s) {
  const size_t n = (size_t)mesh->nfc * D2;
  const int nfc = (int)mesh->nfc;
  double* V = ws;  // basis vector i at V + i n
  double* w = V + (size_t)(m + 1) * n;
  double* z = w + n;
  double* r = z + n;
  double* Minv = r + n;
  double* part = Minv + (size_t)nfc * D2 * D2;
  // small: [0, m + 1) first-pass coefficients, [m + 1, 2m + 2) second-pass ones, [2m + 2] the
  // squared norm; y reuses [0, m)
  double* small = part + (size_t)kMdotBlocks * (m + 2);
  // small: [0, m + 2) first-pass coefficients and, after them, ||w||^2 before the pass;
  // [m + 2, 2m + 4) second-pass coefficients; [2m + 4] ||w||^2 after; y reuses [0, m)
  double* h1 = small;
  double* h2 = small + (m + 2);
  double* nrm = small + 2 * (m + 2);
  const unsigned T = 256;
  const unsigned gr = (unsigned)((n + T - 1) / T);
  const unsigned gv = (unsigned)std::max<size_t>(1, std::min<size_t>((n + T - 1) / T, 8192));
  if (nfc) k_bj_setup_lu<D2><<<(nfc + 63) / 64, 64, 0, s>>>(H, mesh->d_diag, nfc, Minv);
  auto norm2 = [&](const double* a) {
    k_dot_partial<double, double><<<kRedBlocks, kRedThreads, 0, s>>>(a, a, n, part);
    k_dot_final<<<1, kRedThreads, 0, s>>>(part, nrm);
  };
  auto read = [&](const double* d, double* h, int cnt) -> hipError_t {
    hipError_t e = hipMemcpyAsync(h, d, sizeof(double) * cnt, hipMemcpyDeviceToHost, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
  };
  std::vector<double> Hh((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), col(2 * (m + 2) + 1);
  hipError_t e;
  double bn2 = 0;
  norm2(b);
  if ((e = read(nrm, &bn2, 1)) != hipSuccess) return check_hip(e, "hdg_solve_gmres");
  const double bnorm = bn2 > 0 ? std::sqrt(bn2) : 1.0;
  int iters = 0, cycles = 0, reorth = 0;
  double rel = 0;
  for (;;) {
    // true residual at the start of every cycle (and once more at the end)
    if (n) k_residual<D2><<<gr, T, 0, s>>>(mesh->d_row_ptr, mesh->d_col_idx, H, x, b, r, nfc);
    double rn2 = 0;
    norm2(r);
    if ((e = read(nrm, &rn2, 1)) != hipSuccess) return check_hip(e, "hdg_solve_gmres");
    const double beta = std::sqrt(rn2);
    rel = beta / bnorm;
    if (!std::isfinite(rel) || rel <= rtol || iters >= max_iter) break;
    k_scale_into<<<gv, T, 0, s>>>(V, r, nullptr, beta, n);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0;
    bool done = false;
    while (j < m && iters < max_iter && !done) {
      const double* vj = V + (size_t)j * n;
      k_precond<D2, double, double><<<gr, T, 0, s>>>(Minv, vj, z, nfc);
      launch_spmv<D2>(mesh, H, z, w, s);
      // classical Gram-Schmidt against V_0..V_j; a second pass only under severe
      // cancellation, when the first pass left less than 1e-3 of ||w|| (the usual 1/sqrt(2)
      // criterion fires on nearly every Arnoldi step here and doubles the cost, while the
      // iteration counts and the true-residual-checked results are the same without it)
      k_mdot_partial<<<kMdotBlocks, kRedThreads, 0, s>>>(V, n, j + 1, 1, w, n, part);
      k_mdot_final<<<j + 2, kRedThreads, 0, s>>>(part, j + 2, h1, 0);
      k_sub_combination<<<gv, T, 0, s>>>(w, V, n, j + 1, h1, n);
      norm2(w);
      if ((e = read(small, col.data(), 2 * (m + 2) + 1)) != hipSuccess) return check_hip(e, "hdg_solve_gmres");
      for (int i = 0; i <= j; ++i) Hh[(size_t)i * m + j] = col[i];
      double wa2 = col[2 * (m + 2)];
      if (wa2 < 1e-6 * col[j + 1]) {
        k_mdot_partial<<<kMdotBlocks, kRedThreads, 0, s>>>(V, n, j + 1, 0, w, n, part);
        k_mdot_final<<<j + 1, kRedThreads, 0, s>>>(part, j + 1, h2, 0);
        k_sub_combination<<<gv, T, 0, s>>>(w, V, n, j + 1, h2, n);
        norm2(w);
        if ((e = read(small, col.data(), 2 * (m + 2) + 1)) != hipSuccess) return check_hip(e, "hdg_solve_gmres");
        for (int i = 0; i <= j; ++i) Hh[(size_t)i * m + j] += col[m + 2 + i];
        wa2 = col[2 * (m + 2)];
        ++reorth;
      }
      const double hnext = std::sqrt(wa2);
      Hh[(size_t)(j + 1) * m + j] = hnext;
      if (hnext > 0) k_scale_into<<<gv, T, 0, s>>>(V + (size_t)(j + 1) * n, w, nullptr, hnext, n);
      // the earlier Givens rotations, then one that zeroes H(j + 1, j)
      for (int i = 0; i < j; ++i) {
        const double a = Hh[(size_t)i * m + j], c2 = Hh[(size_t)(i + 1) * m + j];
        Hh[(size_t)i * m + j] = cs[i] * a + sn[i] * c2;
        Hh[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c2;
      }
      const double a = Hh[(size_t)j * m + j], c2 = hnext;
      const double den = std::hypot(a, c2);
      cs[j] = den > 0 ? a / den : 1.0;
      sn[j] = den > 0 ? c2 / den : 0.0;
      Hh[(size_t)j * m + j] = den;
      Hh[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++j;
      ++iters;
      // the least-squares residual equals the preconditioned system's residual norm in exact
      // arithmetic; stop the cycle a little early and let the true residual decide
      done = std::fabs(g[j]) <= 0.5 * rtol * bnorm || hnext == 0;
    }
    // y = R^{-1} g by back substitution, then x += M^{-1} (V y)
    for (int i = j - 1; i >= 0; --i) {
      double acc = g[i];
      for (int c = i + 1; c < j; ++c) acc -= Hh[(size_t)i * m + c] * y[c];
      y[i] = Hh[(size_t)i * m + i] != 0 ? acc / Hh[(size_t)i * m + i] : 0.0;
    }
    if ((e = hipMemcpyAsync(small, y.data(), sizeof(double) * j, hipMemcpyHostToDevice, s)) != hipSuccess)
      return check_hip(e, "hdg_solve_gmres");
    k_combination<<<gv, T, 0, s>>>(w, V, n, j, small, n);
    k_precond<D2, double, double><<<gr, T, 0, s>>>(Minv, w, z, nfc);
    k_add_into<<<gv, T, 0, s>>>(x, z, n);
    ++cycles;
  }
  HDG_CHECK_LAUNCH("hdg_solve_gmres");
  info->iterations = iters;
  info->outer = cycles;
  info->rel_residual = rel;
  info->fell_back = reorth;  // GMRES: the number of second Gram-Schmidt passes
  if (!(rel <= rtol)) return set_error(HDG_ERR_NOT_CONVERGED, "hdg_solve_gmres: tolerance not reached");
  return HDG_OK;
}

}  // namespace
}  // namespace hdg

extern "C" hdg_status hdg_solve_gmres_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, int restart,
                                                     size_t* ws_bytes) {
  if (!disc || !mesh || !ws_bytes || restart < 1 || restart > hdg::kMaxRestart)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_solve_gmres_workspace_size: bad argument");
  const int d2 = disc->host.d2;
  *ws_bytes = sizeof(double) * hdg::gmres_ws_doubles((size_t)mesh->nfc * d2, (int)mesh->nfc, d2, restart);
  return HDG_OK;
}

extern "C" hdg_status hdg_solve_gmres(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_H, const double* d_b,
                                      double* d_uhat, double rtol, int max_iter, int restart, hdg_solve_info* info,
                                      void* d_ws, size_t ws_bytes, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_solve_gmres");
  if (st) return st;
  if (!d_H || !d_b || !d_uhat || !info || !(rtol > 0) || max_iter < 0 || restart < 1 ||
      restart > hdg::kMaxRestart)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_solve_gmres: bad argument");
  size_t need = 0;
  hdg_solve_gmres_workspace_size(disc, mesh, restart, &need);
  if (!d_ws || ws_bytes < need) return set_error(HDG_ERR_WORKSPACE, "hdg_solve_gmres: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  double* ws = (double*)d_ws;
  switch (disc->host.k) {
    case 0: return run_gmres<dim2(0)>(mesh, d_H, d_b, d_uhat, rtol, max_iter, restart, info, ws, s);
    case 1: return run_gmres<dim2(1)>(mesh, d_H, d_b, d_uhat, rtol, max_iter, restart, info, ws, s);
    case 2: return run_gmres<dim2(2)>(mesh, d_H, d_b, d_uhat, rtol, max_iter, restart, info, ws, s);
    case 3: return run_gmres<dim2(3)>(mesh, d_H, d_b, d_uhat, rtol, max_iter, restart, info, ws, s);
    case 4: return run_gmres<dim2(4)>(mesh, d_H, d_b, d_uhat, rtol, max_iter, restart, info, ws, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_solve_gmres: unsupported degree");
}

// ---------------------------------------------------------------------------------------
// BiCGStab for the non-symmetric trace system (van der Vorst's stabilised bi-conjugate
// gradients), right-preconditioned by the same block-Jacobi inverses as GMRES: two
// products with H per iteration and short recurrences, so no restart.  The scalars stay
// on the device: scal[0] rho, scal[1] rho_new = (rh, r), scal[2] alpha, scal[3] omega,
// scal[4] (rh, v), scal[5] (t, s), scal[6] (t, t), scal[7] (r, r).  The preconditioner is
// applied inside the vector updates, one face's components meeting in LDS.  Every
// reduction has a fixed order.
namespace hdg {
namespace {

// p = r + beta (p - omega v) (p = r on the first step), ph = Minv p
template <int D2>
__global__ void __launch_bounds__(Lpre<D2>::THREADS) k_bicg_p(const double* __restrict__ r, double* __restrict__ p,
                                                              const double* __restrict__ v,
                                                              const double* __restrict__ Minv, double* __restrict__ ph,
                                                              const double* __restrict__ scal, int first, int nfc) {
  __shared__ double ps[Lpre<D2>::THREADS];
  const int lf = threadIdx.x / D2, c = threadIdx.x % D2;
  const int f = blockIdx.x * Lpre<D2>::FACES + lf;
  const size_t i = (size_t)f * D2 + c;
  double pv = 0.0;
  if (f < nfc) {
    if (first) {
      pv = r[i];
    } else {
      const double beta = (scal[1] / scal[0]) * (scal[2] / scal[3]);
      pv = r[i] + beta * (p[i] - scal[3] * v[i]);
    }
    p[i] = pv;
  }
  ps[threadIdx.x] = pv;
  __syncthreads();
  if (f < nfc) {
    const double* m = Minv + ((size_t)f * D2 + c) * D2;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < D2; ++j) acc += m[j] * ps[lf * D2 + j];
    ph[i] = acc;
  }
}

// alpha = rho_new / (rh, v);  s = r - alpha v,  sh = Minv s
template <int D2>
__global__ void __launch_bounds__(Lpre<D2>::THREADS) k_bicg_s(const double* __restrict__ r,
                                                              const double* __restrict__ v,
                                                              const double* __restrict__ Minv, double* __restrict__ s,
                                                              double* __restrict__ sh, double* __restrict__ scal,
                                                              int nfc) {
  __shared__ double ss[Lpre<D2>::THREADS];
  const int lf = threadIdx.x / D2, c = threadIdx.x % D2;
  const int f = blockIdx.x * Lpre<D2>::FACES + lf;
  const size_t i = (size_t)f * D2 + c;
  const double alpha = scal[1] / scal[4];
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[2] = alpha;  // no thread of this kernel reads it
  double sv = 0.0;
  if (f < nfc) {
    sv = r[i] - alpha * v[i];
    s[i] = sv;
  }
  ss[threadIdx.x] = sv;
  __syncthreads();
  if (f < nfc) {
    const double* m = Minv + ((size_t)f * D2 + c) * D2;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < D2; ++j) acc += m[j] * ss[lf * D2 + j];
    sh[i] = acc;
  }
}

// omega = (t, s) / (t, t);  x += alpha ph + omega sh,  r = s - omega t;  rho <- rho_new
__global__ void k_bicg_xr(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ s,
                          const double* __restrict__ t, const double* __restrict__ ph, const double* __restrict__ sh,
                          double* __restrict__ scal, size_t n) {
  const double alpha = scal[2], omega = scal[5] / scal[6];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    x[i] = x[i] + alpha * ph[i] + omega * sh[i];
    r[i] = s[i] - omega * t[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // no thread of this kernel reads these slots
    scal[3] = omega;
    scal[0] = scal[1];
  }
}

size_t bicg_ws_doubles(size_t n, int nfc, int d2) { return 10 * n + (size_t)nfc * d2 * d2 + kRedBlocks + 16 + 64; }

template <int D2>
hdg_status run_bicgstab(const hdg_mesh* mesh, const double* H, const double* b, double* x, double rtol, int max_iter,
                        int every, hdg_solve_info* info, double* ws, hipStream_t s) {
  const size_t n = (size_t)mesh->nfc * D2;
  const int nfc = (int)mesh->nfc;
  double* r = ws;
  double* rh = r + n;
  double* p = rh + n;
  double* ph = p + n;
  double* v = ph + n;
  double* sv = v + n;
  double* sh = sv + n;
  double* t = sh + n;
  double* xs = t + n;  // the last iterate whose residual was finite
  double* Minv = xs + n + n;
  double* part = Minv + (size_t)nfc * D2 * D2;
  double* scal = part + kRedBlocks;
  const unsigned T = 256;
  const unsigned gr = (unsigned)((n + T - 1) / T);
  const unsigned gv = (unsigned)std::max<size_t>(1, std::min<size_t>((n + T - 1) / T, 8192));
  const unsigned gf = (unsigned)((nfc + Lpre<D2>::FACES - 1) / Lpre<D2>::FACES);
  constexpr unsigned TL = Lpre<D2>::THREADS;
  auto dot = [&](const double* a, const double* c, double* out) {
    k_dot_partial<double, double><<<kRedBlocks, kRedThreads, 0, s>>>(a, c, n, part);
    k_dot_final<<<1, kRedThreads, 0, s>>>(part, out);
  };
  auto read = [&](const double* d) -> double {
    double h = 0;
    if (hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return std::nan("");
    if (hipStreamSynchronize(s) != hipSuccess) return std::nan("");
    return h;
  };
  k_bj_setup_lu<D2><<<(nfc + 63) / 64, 64, 0, s>>>(H, mesh->d_diag, nfc, Minv);
  dot(b, b, scal + 8);
  const double bb = read(scal + 8);
  HDG_CHECK_LAUNCH("hdg_solve_bicgstab setup");
  info->iterations = 0;
  info->outer = 0;
  info->fell_back = 0;
  info->rel_residual = 0;
  if (!(bb > 0)) {
    k_fill<double><<<gv, T, 0, s>>>(x, n, 0.0);
    return HDG_OK;
  }
  const double tol2 = rtol * rtol * bb;
  int it = 0, restarts = 0;
  auto restart = [&]() {  // the true residual, a new shadow vector, and a first step
    k_residual<D2><<<gr, T, 0, s>>>(mesh->d_row_ptr, mesh->d_col_idx, H, x, b, r, nfc);
    k_copy<double><<<gv, T, 0, s>>>(r, rh, n);
    k_copy<double><<<gv, T, 0, s>>>(x, xs, n);
  };
  restart();
  bool first = true;
  for (;;) {
    if (it % every == 0 || it >= max_iter) {
      dot(r, r, scal + 7);
      const double rr = read(scal + 7);
      HDG_CHECK_LAUNCH("hdg_solve_bicgstab");
      if (!std::isfinite(rr)) {  // breakdown: back to the last finite iterate
        if (restarts >= 50) break;
        k_copy<double><<<gv, T, 0, s>>>(xs, x, n);
        restart();
        first = true;
        ++restarts;
        continue;
      }
      k_copy<double><<<gv, T, 0, s>>>(x, xs, n);
      if (rr <= tol2 || it >= max_iter) {
        k_residual<D2><<<gr, T, 0, s>>>(mesh->d_row_ptr, mesh->d_col_idx, H, x, b, r, nfc);
        dot(r, r, scal + 7);
        const double tr = read(scal + 7);
        info->iterations = it;
        info->outer = restarts;
        info->rel_residual = std::sqrt(tr / bb);
        if (tr <= tol2) return HDG_OK;
        if (it >= max_iter) return set_error(HDG_ERR_NOT_CONVERGED, "hdg_solve_bicgstab: iteration limit reached");
        restart();  // the recursive residual drifted from the true one
        first = true;
        ++restarts;
      }
    }
    dot(rh, r, scal + 1);
    k_bicg_p<D2><<<gf, TL, 0, s>>>(r, p, v, Minv, ph, scal, first ? 1 : 0, nfc);
    launch_spmv<D2>(mesh, H, ph, v, s);
    dot(rh, v, scal + 4);
    k_bicg_s<D2><<<gf, TL, 0, s>>>(r, v, Minv, sv, sh, scal, nfc);
    launch_spmv<D2>(mesh, H, sh, t, s);
    dot(t, sv, scal + 5);
    dot(t, t, scal + 6);
    k_bicg_xr<<<gv, T, 0, s>>>(x, r, sv, t, ph, sh, scal, n);
    first = false;
    ++it;
  }
  info->iterations = it;
  info->outer = restarts;
  info->rel_residual = std::nan("");
  return set_error(HDG_ERR_NOT_CONVERGED, "hdg_solve_bicgstab: repeated breakdown");
}

}  // namespace
}  // namespace hdg

extern "C" hdg_status hdg_solve_bicgstab_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, size_t* ws_bytes) {
  if (!disc || !mesh || !ws_bytes) return set_error(HDG_ERR_INVALID_ARG, "hdg_solve_bicgstab_workspace_size: NULL");
  const int d2 = disc->host.d2;
  *ws_bytes = sizeof(double) * hdg::bicg_ws_doubles((size_t)mesh->nfc * d2, (int)mesh->nfc, d2);
  return HDG_OK;
}

extern "C" hdg_status hdg_solve_bicgstab(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_H,
                                         const double* d_b, double* d_uhat, double rtol, int max_iter, int check_every,
                                         hdg_solve_info* info, void* d_ws, size_t ws_bytes, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_solve_bicgstab");
  if (st) return st;
  if (!d_H || !d_b || !d_uhat || !info || !(rtol > 0) || max_iter < 0 || check_every < 1)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_solve_bicgstab: bad argument");
  size_t need = 0;
  hdg_solve_bicgstab_workspace_size(disc, mesh, &need);
  if (!d_ws || ws_bytes < need) return set_error(HDG_ERR_WORKSPACE, "hdg_solve_bicgstab: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  double* ws = (double*)d_ws;
  switch (disc->host.k) {
    case 0: return run_bicgstab<dim2(0)>(mesh, d_H, d_b, d_uhat, rtol, max_iter, check_every, info, ws, s);
    case 1: return run_bicgstab<dim2(1)>(mesh, d_H, d_b, d_uhat, rtol, max_iter, check_every, info, ws, s);
    case 2: return run_bicgstab<dim2(2)>(mesh, d_H, d_b, d_uhat, rtol, max_iter, check_every, info, ws, s);
    case 3: return run_bicgstab<dim2(3)>(mesh, d_H, d_b, d_uhat, rtol, max_iter, check_every, info, ws, s);
    case 4: return run_bicgstab<dim2(4)>(mesh, d_H, d_b, d_uhat, rtol, max_iter, check_every, info, ws, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_solve_bicgstab: unsupported degree");
}
