// Learned face-graph preconditioner for the trace system H uhat = b (eq 6.5; the paper
// leaves the solver open).
//
// Scaled system.  With H_ii = L_i L_i^T, Hs_ij = L_i^{-1} H_ij L_j^{-T} (so Hs_ii = I).
// Preconditioner.  M^{-1} = L^{-T} G^T G L^{-1}, G = B (I + N), N strictly block-lower on the
// pattern of H, B block diagonal with lower-triangular blocks of positive diagonal.  It is
// symmetric positive definite for every N and B.
// Network (FP32).  One node per face and one edge per off-diagonal block.  Node features
// are the one-hot face type, log(|e| nfc^{2/3}) and the row energy sum_j ||Hs_ij||_F^2.
// Edge features are the entries of Hs_ij.  The layers, with relu activations:
//     X = relu(W0 a + c0),  E = relu(We b + ce),
//     M_ij = relu(Wm_l [X_i; X_j; E_ij] + cm_l),  X_i += relu(Wu_l [X_i; sum_j M_ij] + cu_l)
// and the heads, N on the lower edges with no Dirichlet face and beta on the other faces:
//     N_ij = -Hs_ij + reshape(Wo [X_i; X_j; E_ij] + co),   beta_i = Wb X_i + cb,
// B_i[a][a] = exp(beta_i[a]), B_i[a][b] = beta_i[d2 + a (a - 1) / 2 + b] (b < a).
// Objective.  The logarithm of the Kaporin number (tr/n) / det^{1/n} of G Hs G^T, with
// det(G Hs G^T) = det(B)^2 det(Hs):  loss = log T - (2/n) sum_i sum_a beta_i[a],
// T = 1/(p n) sum_z (G^T z)^T Hs (G^T z) over probe vectors z.
//
// Kernel layout.  Every layer is a row-wise dense product over gathered, concatenated
// inputs (one thread per output entry; the weights sit transposed in LDS, so that the
// lanes of a wavefront read consecutive words).  Sums over the edges of a face are
// segmented sums over its CSR row, in row order.  Sums into the column face of an edge go
// through the mirror index (the position of block (j, i)), over the row of the
// receiving face.  No atomics are used, so every run gives the same bits.  Weight
// gradients are two-stage reductions with fixed chunks, accumulated in FP64.
#include <cmath>
#include <vector>

#include "device_common.h"

namespace hdg {
namespace {

constexpr int kF0 = 5;        // node features
constexpr int kWgChunks = 120;  // row chunks of the weight-gradient reduction

enum SelMode { SEL_ALL = 0, SEL_OFF = 1, SEL_HEAD = 2, SEL_FREE = 3 };

__device__ __forceinline__ bool selected(int mode, int r, const int* erow, const int* col, const int* ftype) {
  if (mode == SEL_ALL) return true;
  if (mode == SEL_FREE) return ftype[r] != 1;  // node rows: every face but a Dirichlet one
  const int i = erow[r], j = col[r];
  if (mode == SEL_OFF) return i != j;
  return j < i && ftype[i] != 1 && ftype[j] != 1;
}

struct Seg {
  const float* src;
  const int* gidx;  // row r reads src[gidx[r] * width + k] (identity if null)
  int width;
};

struct Segs {
  Seg s[3];
  int n;
  int nin;
};

__device__ __forceinline__ float seg_in(const Segs& in, int r, int k) {
  int o = 0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (q < in.n) {
      const Seg& sg = in.s[q];
      if (k < o + sg.width) {
        const int row = sg.gidx ? sg.gidx[r] : r;
        return sg.src[(size_t)row * sg.width + (k - o)];
      }
      o += sg.width;
    }
  }
  return 0.0f;
}

// out[r][o] = sel(r) ? act(b[o] + sum_k W[o][k] in(r, k)) (+ resid[r][o]) : 0;
// head form: out = sel(r) ? acc - sub[r][o] : 0.  pre (optional) keeps the pre-activation.
__global__ void k_dense(int R, Segs in, const float* __restrict__ W, const float* __restrict__ b, int nout, int act,
                        const float* __restrict__ resid, const float* __restrict__ sub, float* __restrict__ pre,
                        float* __restrict__ out, int mode, const int* __restrict__ erow, const int* __restrict__ col,
                        const int* __restrict__ ftype) {
  extern __shared__ float s_wt[];  // [nin][nout] transposed weights
  const int nin = in.nin;
  for (int t = threadIdx.x; t < nin * nout; t += blockDim.x) {
    const int o = t / nin, k = t % nin;
    s_wt[k * nout + o] = W[t];
  }
  __syncthreads();
  const size_t total = (size_t)R * nout;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx / nout), o = (int)(idx % nout);
    float v = 0.0f;
    if (selected(mode, r, erow, col, ftype)) {
      float acc = b[o];
      for (int k = 0; k < nin; ++k) acc = fmaf(s_wt[k * nout + o], seg_in(in, r, k), acc);
      if (pre) pre[idx] = acc;
      if (sub) {
        v = acc - sub[idx];
      } else {
        v = act ? fmaxf(acc, 0.0f) : acc;
        if (resid) v += resid[idx];
      }
    } else if (pre) {
      pre[idx] = 0.0f;
    }
    out[idx] = v;
  }
}

// The same layer on the FP32 matrix cores (v_mfma_f32_16x16x4f32): each wavefront takes 16
// rows and all NT x 16 outputs; per step of 4 inputs a lane gathers one input value
// (row = lane % 16, input = lane / 16) and the MFMA multiplies it against the transposed
// weights in LDS (zero-padded to NT x 16 outputs and a multiple of 4 inputs).  The
// accumulator of tile nt holds rows 4 (lane / 16) + i and output nt * 16 + lane % 16.
// Same epilogue as k_dense.
typedef float v4f __attribute__((ext_vector_type(4)));

template <int NT>
__global__ void __launch_bounds__(256) k_dense_mfma(int R, Segs in, const float* __restrict__ W,
                                                    const float* __restrict__ b, int nout, int act,
                                                    const float* __restrict__ resid, const float* __restrict__ sub,
                                                    float* __restrict__ pre, float* __restrict__ out, int mode,
                                                    const int* __restrict__ erow, const int* __restrict__ col,
                                                    const int* __restrict__ ftype) {
  constexpr int NP = NT * 16;
  extern __shared__ float s_wt[];  // [kp][NP] transposed weights, then the bias [NP]
  const int nin = in.nin, kp = (nin + 3) & ~3;
  float* s_b = s_wt + kp * NP;
  for (int t = threadIdx.x; t < kp * NP; t += blockDim.x) {
    const int k = t / NP, o = t % NP;
    s_wt[t] = (k < nin && o < nout) ? W[(size_t)o * nin + k] : 0.0f;
  }
  for (int t = threadIdx.x; t < NP; t += blockDim.x) s_b[t] = t < nout ? b[t] : 0.0f;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int tiles = (R + 15) / 16;
  for (int tile = blockIdx.x * 4 + wave; tile < tiles; tile += gridDim.x * 4) {
    const int ra = tile * 16 + r16;  // the row this lane feeds to the A operand
    v4f acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < kp; kk += 4) {
      const int k = kk + k4;
      const float a = (ra < R && k < nin) ? seg_in(in, ra, k) : 0.0f;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, s_wt[k * NP + nt * 16 + r16], acc[nt], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = tile * 16 + 4 * k4 + i;
      if (r >= R) continue;
      const bool sel = selected(mode, r, erow, col, ftype);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int o = nt * 16 + r16;
        if (o >= nout) continue;
        const size_t idx = (size_t)r * nout + o;
        float v = 0.0f;
        if (sel) {
          const float pa = acc[nt][i] + s_b[o];
          if (pre) pre[idx] = pa;
          if (sub) {
            v = pa - sub[idx];
          } else {
            v = act ? fmaxf(pa, 0.0f) : pa;
            if (resid) v += resid[idx];
          }
        } else if (pre) {
          pre[idx] = 0.0f;
        }
        out[idx] = v;
      }
    }
  }
}

// out[r][k] = (resid ? resid[r][k] : 0) + sum_o W[o][koff + k] d[r][o]   (k < width)
__global__ void k_dense_t(int R, const float* __restrict__ W, int nin, int nout, int koff, int width,
                          const float* __restrict__ d, const float* __restrict__ resid, float* __restrict__ out) {
  extern __shared__ float s_w[];  // [nout][width]
  for (int t = threadIdx.x; t < nout * width; t += blockDim.x) {
    const int o = t / width, k = t % width;
    s_w[t] = W[(size_t)o * nin + koff + k];
  }
  __syncthreads();
  const size_t total = (size_t)R * width;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx / width), k = (int)(idx % width);
    float acc = resid ? resid[idx] : 0.0f;
    const float* dr = d + (size_t)r * nout;
    for (int o = 0; o < nout; ++o) acc = fmaf(s_w[o * width + k], dr[o], acc);
    out[idx] = acc;
  }
}

// Segmented sums over the CSR rows: out[i][c] (+)= sum_{e in row i} t[e'][c] with
// e' = e (own edges) or mirror[e] (edges whose column is i), for selected e'.
__global__ void k_rowsum(int nfc, int width, const int* __restrict__ row_ptr, const int* __restrict__ mirror,
                         const float* __restrict__ t, float* __restrict__ out, int accumulate, int mode,
                         const int* __restrict__ erow, const int* __restrict__ col, const int* __restrict__ ftype) {
  const size_t total = (size_t)nfc * width;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / width), c = (int)(idx % width);
    float acc = accumulate ? out[idx] : 0.0f;
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int ep = mirror ? mirror[e] : e;
      if (selected(mode, ep, erow, col, ftype)) acc += t[(size_t)ep * width + c];
    }
    out[idx] = acc;
  }
}

// d[r][c] = g[gidx ? gidx[r] : r][c] * (pre[r][c] > 0), zero on unselected rows.
__global__ void k_relu_grad(int R, int width, const float* __restrict__ g, const int* __restrict__ gidx,
                            const float* __restrict__ pre, float* __restrict__ d, int mode, const int* __restrict__ erow,
                            const int* __restrict__ col, const int* __restrict__ ftype) {
  const size_t total = (size_t)R * width;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx / width), c = (int)(idx % width);
    float v = 0.0f;
    if (selected(mode, r, erow, col, ftype) && pre[idx] > 0.0f) v = g[(size_t)(gidx ? gidx[r] : r) * width + c];
    d[idx] = v;
  }
}

// Weight gradient, stage 1: part[chunk][o][k] = sum_{r in chunk} d[r][o] in(r, k), with
// in(r, nin) = 1 (bias).  One thread per (o, k).
__global__ void k_wgrad_partial(int R, Segs in, const float* __restrict__ d, int nout, double* __restrict__ part) {
  const int nin = in.nin, P = nout * (nin + 1);
  const int pid = blockIdx.y * blockDim.x + threadIdx.x;
  const int chunk = (R + kWgChunks - 1) / kWgChunks;
  const int r0 = blockIdx.x * chunk, r1 = min(R, r0 + chunk);
  if (pid >= P) return;
  const int o = pid / (nin + 1), k = pid % (nin + 1);
  double acc = 0.0;
  for (int r = r0; r < r1; ++r) {
    const float dv = d[(size_t)r * nout + o];
    if (dv != 0.0f) acc += (double)dv * (k < nin ? (double)seg_in(in, r, k) : 1.0);
  }
  part[(size_t)blockIdx.x * P + pid] = acc;
}

// Stage 2: gradW[o][k] and gradb[o] = sum over the chunks in order.
__global__ void k_wgrad_final(int nout, int nin, const double* __restrict__ part, float* __restrict__ gW,
                              float* __restrict__ gb) {
  const int P = nout * (nin + 1);
  const int pid = blockIdx.x * blockDim.x + threadIdx.x;
  if (pid >= P) return;
  double s = 0.0;
  for (int c = 0; c < kWgChunks; ++c) s += part[(size_t)c * P + pid];
  const int o = pid / (nin + 1), k = pid % (nin + 1);
  if (k < nin)
    gW[(size_t)o * nin + k] = (float)s;
  else
    gb[o] = (float)s;
}

// ---- graph set-up

__global__ void k_erow(int nfc, const int* __restrict__ row_ptr, int* __restrict__ erow) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfc) return;
  for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) erow[e] = i;
}

template <int D2>
__device__ void chol_inv(const double* __restrict__ A, double (&Li)[D2][D2]) {
  double L[D2][D2] = {};
  for (int i = 0; i < D2; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = A[i * D2 + j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      L[i][j] = (i == j) ? sqrt(s) : s / L[j][j];
    }
  for (int j = 0; j < D2; ++j)
    for (int i = 0; i < D2; ++i) {
      if (i < j) {
        Li[i][j] = 0.0;
        continue;
      }
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= L[i][k] * Li[k][j];
      Li[i][j] = s / L[i][i];
    }
}

template <int D2>
__global__ void k_gnn_diag(int nfc, const int* __restrict__ diag, const double* __restrict__ H,
                           double* __restrict__ Linv64, float* __restrict__ Linv32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfc) return;
  double Li[D2][D2];
  chol_inv<D2>(H + (size_t)diag[i] * D2 * D2, Li);
  for (int a = 0; a < D2; ++a)
    for (int b = 0; b < D2; ++b) {
      Linv64[((size_t)i * D2 + a) * D2 + b] = Li[a][b];
      Linv32[((size_t)i * D2 + a) * D2 + b] = (float)Li[a][b];
    }
}

// Hs_e = Linv_i H_e Linv_j^T, mirror[e] = position of (j, i) in row j (columns ascending)
template <int D2>
__global__ void k_gnn_edges(int nnzb, const int* __restrict__ row_ptr, const int* __restrict__ col,
                            const int* __restrict__ erow, const double* __restrict__ H,
                            const double* __restrict__ Linv, float* __restrict__ Hs, int* __restrict__ mirror) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnzb) return;
  const int i = erow[e], j = col[e];
  const double* Li = Linv + (size_t)i * D2 * D2;
  const double* Lj = Linv + (size_t)j * D2 * D2;
  const double* He = H + (size_t)e * D2 * D2;
  double T[D2][D2];
  for (int a = 0; a < D2; ++a)
    for (int b = 0; b < D2; ++b) {
      double s = 0.0;
      for (int c = 0; c <= a; ++c) s += Li[a * D2 + c] * He[c * D2 + b];
      T[a][b] = s;
    }
  for (int a = 0; a < D2; ++a)
    for (int b = 0; b < D2; ++b) {
      double s = 0.0;
      for (int c = 0; c <= b; ++c) s += T[a][c] * Lj[b * D2 + c];
      Hs[((size_t)e * D2 + a) * D2 + b] = (float)s;
    }
  int lo = row_ptr[j], hi = row_ptr[j + 1] - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (col[mid] < i) lo = mid + 1; else hi = mid;
  }
  mirror[e] = lo;
}

__global__ void k_gnn_nodes(int nfc, int fe, const int* __restrict__ row_ptr, const int* __restrict__ col,
                            const int* __restrict__ ftype, const double* __restrict__ area, double area_scale,
                            const float* __restrict__ Hs, float* __restrict__ node) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfc) return;
  double en = 0.0;
  for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    if (col[e] == i) continue;
    for (int q = 0; q < fe; ++q) {
      const double v = Hs[(size_t)e * fe + q];
      en += v * v;
    }
  }
  float* a = node + (size_t)i * kF0;
  const int t = ftype[i];
  a[0] = t == 0 ? 1.0f : 0.0f;
  a[1] = t == 1 ? 1.0f : 0.0f;
  a[2] = t == 2 ? 1.0f : 0.0f;
  a[3] = (float)log(area[i] * area_scale);
  a[4] = (float)en;
}

// ---- probe loss: y = B^T z, u = (I + N)^T y, hu = Hs u, T = sum u.hu / (p n),
// loss = log T - (2/n) sum beta_diag;  dT/dN_e = 2/(p n) sum_z y_i hu_j^T,
// dT/dB_i[a][b] = 2/(p n) sum_z z_i[a] w_i[b] with w = (I + N) hu.

__device__ __forceinline__ int tri_pair_a(int q) {  // q = a (a - 1) / 2 + b, b < a  ->  a
  int a = 1;
  while ((a + 1) * a / 2 <= q) ++a;
  return a;
}

// y_i[b] = sum_{a >= b} B_i[a][b] z_i[a]
__global__ void k_apply_BT(int nfc, int d2, int np, const float* __restrict__ Bp, const float* __restrict__ z,
                           float* __restrict__ y) {
  const size_t n = (size_t)nfc * d2, total = n * np;
  const int fb = d2 * (d2 + 1) / 2;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const size_t p = idx / n, rem = idx % n;
    const int i = (int)(rem / d2), b = (int)(rem % d2);
    const float* bp = Bp + (size_t)i * fb;
    const float* zi = z + p * n + (size_t)i * d2;
    float acc = expf(bp[b]) * zi[b];
    for (int a = b + 1; a < d2; ++a) acc = fmaf(bp[d2 + a * (a - 1) / 2 + b], zi[a], acc);
    y[idx] = acc;
  }
}

// w_i = hu_i + sum_{e in row i, col(e) < i} N_e hu_{col(e)}
__global__ void k_apply_G(int nfc, int d2, int np, const int* __restrict__ row_ptr, const int* __restrict__ col,
                          const float* __restrict__ N, const float* __restrict__ hu, float* __restrict__ w) {
  const size_t n = (size_t)nfc * d2, total = n * np;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const size_t p = idx / n, rem = idx % n;
    const int i = (int)(rem / d2), a = (int)(rem % d2);
    const float* hp = hu + p * n;
    float acc = hp[rem];
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int j = col[e];
      if (j >= i) break;  // columns ascend
      const float* Na = N + ((size_t)e * d2 + a) * d2;
      for (int b = 0; b < d2; ++b) acc = fmaf(Na[b], hp[(size_t)j * d2 + b], acc);
    }
    w[idx] = acc;
  }
}


// u_j = z_j + sum_{e' in row j, col(e') > j} N_{mirror(e')}^T z_{col(e')}
__global__ void k_apply_GT(int nfc, int d2, int np, const int* __restrict__ row_ptr, const int* __restrict__ col,
                           const int* __restrict__ mirror, const float* __restrict__ N, const float* __restrict__ z,
                           float* __restrict__ u) {
  const size_t n = (size_t)nfc * d2, total = n * np;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const size_t p = idx / n, rem = idx % n;
    const int j = (int)(rem / d2), a = (int)(rem % d2);
    const float* zp = z + p * n;
    float acc = zp[rem];
    for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e) {
      const int i = col[e];
      if (i <= j) continue;
      const float* Nb = N + (size_t)mirror[e] * d2 * d2;  // block N_ij
      for (int b = 0; b < d2; ++b) acc = fmaf(Nb[b * d2 + a], zp[(size_t)i * d2 + b], acc);
    }
    u[idx] = acc;
  }
}

__global__ void k_spmv_hs(int nfc, int d2, int np, const int* __restrict__ row_ptr, const int* __restrict__ col,
                          const float* __restrict__ Hs, const float* __restrict__ u, float* __restrict__ hu) {
  const size_t n = (size_t)nfc * d2, total = n * np;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const size_t p = idx / n, rem = idx % n;
    const int i = (int)(rem / d2), a = (int)(rem % d2);
    const float* up = u + p * n;
    float acc = 0.0f;
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const float* B = Hs + ((size_t)e * d2 + a) * d2;
      const float* uj = up + (size_t)col[e] * d2;
      for (int b = 0; b < d2; ++b) acc = fmaf(B[b], uj[b], acc);
    }
    hu[idx] = acc;
  }
}

constexpr int kRedB = 256, kRedT = 256;

__global__ void k_dot_part(const float* __restrict__ a, const float* __restrict__ b, size_t n,
                           double* __restrict__ part) {
  __shared__ double sh[kRedT];
  double s = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    s += (double)a[i] * (double)b[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kRedT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_dot_fin(const double* __restrict__ part, double scale, double* __restrict__ out) {
  __shared__ double sh[kRedT];
  double s = 0.0;
  for (int i = threadIdx.x; i < kRedB; i += blockDim.x) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kRedT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] * scale;
}

// The upper position (j, i), i > j, of the factor receives N_ij^T (from its mirror (i, j)),
// so that the transposed sweep of the preconditioner reads block rows contiguously.
__global__ void k_mirror_upper(int nnzb, int d2, const int* __restrict__ erow, const int* __restrict__ col,
                               const int* __restrict__ mirror, float* __restrict__ N) {
  const int fe = d2 * d2;
  const size_t total = (size_t)nnzb * fe;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int e = (int)(idx / fe), q = (int)(idx % fe), a = q / d2, b = q % d2;
    if (col[e] > erow[e]) N[idx] = N[(size_t)mirror[e] * fe + b * d2 + a];
  }
}

// part[block] = partial sums of beta_i[a], a < d2 (the log-diagonal of B)
__global__ void k_logdiag_part(int nfc, int d2, const float* __restrict__ Bp, double* __restrict__ part) {
  __shared__ double sh[kRedT];
  const int fb = d2 * (d2 + 1) / 2;
  const size_t n = (size_t)nfc * d2;
  double s = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    s += (double)Bp[(i / d2) * fb + i % d2];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kRedT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out = log T - c sum(part)
__global__ void k_loss_fin(const double* __restrict__ part, const double* __restrict__ T, double c,
                           double* __restrict__ out) {
  __shared__ double sh[kRedT];
  double s = 0.0;
  for (int i = threadIdx.x; i < kRedB; i += blockDim.x) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kRedT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = log(*T) - c * sh[0];
}

// dbeta_i[q] (free faces; zero on Dirichlet faces), with S = scale / T:
//   q < d2:  S sum_p z_p[i][q] w_p[i][q] exp(beta_i[q]) - c
//   q >= d2 (entry (a, b) of the strict lower triangle):  S sum_p z_p[i][a] w_p[i][b]
__global__ void k_dbeta(int nfc, int d2, int np, size_t n, const int* __restrict__ ftype, const float* __restrict__ Bp,
                        const float* __restrict__ z, const float* __restrict__ w, const double* __restrict__ T,
                        double scale, double c, float* __restrict__ dB) {
  const int fb = d2 * (d2 + 1) / 2;
  const size_t total = (size_t)nfc * fb;
  const double S = scale / *T;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / fb), q = (int)(idx % fb);
    float v = 0.0f;
    if (ftype[i] != 1) {
      int a = q, b = q;
      if (q >= d2) {
        a = tri_pair_a(q - d2);
        b = q - d2 - a * (a - 1) / 2;
      }
      double s = 0.0;
      for (int p = 0; p < np; ++p) s += (double)z[p * n + (size_t)i * d2 + a] * (double)w[p * n + (size_t)i * d2 + b];
      v = q < d2 ? (float)(S * s * exp((double)Bp[idx]) - c) : (float)(S * s);
    }
    dB[idx] = v;
  }
}

// dD[e][a*d2+b] = sel_head(e) ? (scale / T) sum_p y_p[i][a] hu_p[j][b] : 0
__global__ void k_dN(int nnzb, int d2, int np, size_t n, const int* __restrict__ erow, const int* __restrict__ col,
                     const int* __restrict__ ftype, const float* __restrict__ z, const float* __restrict__ hu,
                     const double* __restrict__ T, double scale0, float* __restrict__ dD) {
  const double scale = scale0 / *T;
  const int fe = d2 * d2;
  const size_t total = (size_t)nnzb * fe;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int e = (int)(idx / fe), q = (int)(idx % fe), a = q / d2, b = q % d2;
    float v = 0.0f;
    if (selected(SEL_HEAD, e, erow, col, ftype)) {
      const int i = erow[e], j = col[e];
      double s = 0.0;
      for (int p = 0; p < np; ++p) s += (double)z[p * n + (size_t)i * d2 + a] * (double)hu[p * n + (size_t)j * d2 + b];
      v = (float)(scale * s);
    }
    dD[idx] = v;
  }
}

__global__ void k_adam(int64_t n, float* __restrict__ x, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  x[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---- host side

struct Layout {
  int64_t W0, c0, We, ce, Wo, co, Wb, cb, total;
  std::vector<int64_t> Wm, cm, Wu, cu;
};

Layout layout(const hdg_gnn_shape& s) {
  const int h = s.hidden, fe = s.d2 * s.d2;
  Layout L;
  int64_t o = 0;
  auto take = [&](int64_t n) {
    int64_t r = o;
    o += n;
    return r;
  };
  L.W0 = take((int64_t)h * kF0);
  L.c0 = take(h);
  L.We = take((int64_t)h * fe);
  L.ce = take(h);
  for (int l = 0; l < s.layers; ++l) {
    L.Wm.push_back(take((int64_t)h * 3 * h));
    L.cm.push_back(take(h));
    L.Wu.push_back(take((int64_t)h * 2 * h));
    L.cu.push_back(take(h));
  }
  L.Wo = take((int64_t)fe * 3 * h);
  L.co = take(fe);
  const int fb = s.d2 * (s.d2 + 1) / 2;
  L.Wb = take((int64_t)fb * h);
  L.cb = take(fb);
  L.total = o;
  return L;
}

hdg_status check_shape(const hdg_gnn_shape* s, const char* who) {
  if (!s || s->hidden < 1 || s->hidden > 64 || s->layers < 0 || s->layers > 8 ||
      (s->d2 != 1 && s->d2 != 3 && s->d2 != 6 && s->d2 != 10 && s->d2 != 15))
    return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": shape needs d2 in {1,3,6,10,15}, hidden 1..64, "
                                                             "layers 0..8");
  return HDG_OK;
}

struct Carve {
  char* p;
  size_t left;
  bool ok = true;
  template <class T>
  T* take(size_t n) {
    const size_t bytes = (n * sizeof(T) + 255) & ~size_t(255);
    if (bytes > left) {
      ok = false;
      return nullptr;
    }
    T* r = reinterpret_cast<T*>(p);
    p += bytes;
    left -= bytes;
    return r;
  }
};

// Workspace arrays of the forward pass (train adds the backward's).
struct Work {
  std::vector<float*> X, V, Agg, U;
  float *Eh, *M, *dX, *dXin, *dEh, *dV, *t, *dD, *dB, *u, *hu, *y, *wv;
  double *part, *wpart, *loss;
};

size_t work_bytes(const hdg_gnn_shape& s, int64_t nfc, int64_t nnzb, int nprobe, bool carve_only, Work* w,
                  void* ws, size_t ws_bytes, bool* ok) {
  const size_t h = s.hidden, fe = (size_t)s.d2 * s.d2, L = s.layers;
  size_t total = 0;
  Carve cv{(char*)ws, ws_bytes};
  auto F = [&](size_t n) -> float* {
    total += (n * 4 + 255) & ~size_t(255);
    return carve_only ? cv.take<float>(n) : nullptr;
  };
  auto D = [&](size_t n) -> double* {
    total += (n * 8 + 255) & ~size_t(255);
    return carve_only ? cv.take<double>(n) : nullptr;
  };
  Work tmp;
  Work& W = w ? *w : tmp;
  W.X.clear();
  W.V.clear();
  W.Agg.clear();
  W.U.clear();
  for (size_t l = 0; l <= L; ++l) W.X.push_back(F(nfc * h));
  for (size_t l = 0; l < L; ++l) {
    W.V.push_back(F(nnzb * h));
    W.Agg.push_back(F(nfc * h));
    W.U.push_back(F(nfc * h));
  }
  W.Eh = F(nnzb * h);
  W.M = F(nnzb * h);
  W.dX = F(nfc * h);
  W.dXin = F(nfc * h);
  W.dEh = F(nnzb * h);
  W.dV = F(nnzb * h);
  W.t = F(nnzb * h);
  W.dD = F(nnzb * fe);
  W.dB = F(nfc * (size_t)s.d2 * (s.d2 + 1) / 2);
  const size_t np = (size_t)std::max(nprobe, 1);
  W.u = F(np * nfc * s.d2);
  W.hu = F(np * nfc * s.d2);
  W.y = F(np * nfc * s.d2);
  W.wv = F(np * nfc * s.d2);
  W.part = D(kRedB);
  W.loss = D(8);
  size_t maxp = (size_t)h * (kF0 + 1);
  maxp = std::max(maxp, (size_t)h * (fe + 1));
  maxp = std::max(maxp, (size_t)h * (3 * h + 1));
  maxp = std::max(maxp, (size_t)h * (2 * h + 1));
  maxp = std::max(maxp, fe * (3 * h + 1));
  maxp = std::max(maxp, (size_t)s.d2 * (s.d2 + 1) / 2 * (h + 1));
  W.wpart = D((size_t)kWgChunks * maxp);
  if (ok) *ok = cv.ok;
  return total;
}

struct Ctx {
  hipStream_t s;
  int64_t nfc, nnzb;
  const hdg_mesh* mesh;
  const hdg_gnn_graph* g;
  const int* erow() const { return g->erow; }
  const int* col() const { return mesh->d_col_idx; }
  const int* ftype() const { return mesh->d_ftype; }
};

unsigned grid_for(size_t total) { return (unsigned)std::max<size_t>(1, std::min<size_t>((total + 255) / 256, 16384)); }

hdg_status dense(const Ctx& c, int R, const Segs& in, const float* W, const float* b, int nout, int act,
                 const float* resid, const float* sub, float* pre, float* out, int mode) {
  if (nout <= 64) {  // the matrix-core form: 16-row tiles, up to four 16-output tiles
    const int nt = (nout + 15) / 16, kp = (in.nin + 3) & ~3;
    const size_t lds = ((size_t)kp * nt * 16 + nt * 16) * sizeof(float);
    const unsigned grid = (unsigned)std::max(1, std::min((R + 63) / 64, 8192));
    switch (nt) {
      case 1: k_dense_mfma<1><<<grid, 256, lds, c.s>>>(R, in, W, b, nout, act, resid, sub, pre, out, mode, c.erow(), c.col(), c.ftype()); break;
      case 2: k_dense_mfma<2><<<grid, 256, lds, c.s>>>(R, in, W, b, nout, act, resid, sub, pre, out, mode, c.erow(), c.col(), c.ftype()); break;
      case 3: k_dense_mfma<3><<<grid, 256, lds, c.s>>>(R, in, W, b, nout, act, resid, sub, pre, out, mode, c.erow(), c.col(), c.ftype()); break;
      default: k_dense_mfma<4><<<grid, 256, lds, c.s>>>(R, in, W, b, nout, act, resid, sub, pre, out, mode, c.erow(), c.col(), c.ftype()); break;
    }
    HDG_CHECK_LAUNCH("k_dense_mfma");
    return HDG_OK;
  }
  const size_t lds = (size_t)in.nin * nout * sizeof(float);
  k_dense<<<grid_for((size_t)R * nout), 256, lds, c.s>>>(R, in, W, b, nout, act, resid, sub, pre, out, mode,
                                                           c.erow(), c.col(), c.ftype());
  HDG_CHECK_LAUNCH("k_dense");
  return HDG_OK;
}

hdg_status dense_t(const Ctx& c, int R, const float* W, int nin, int nout, int koff, int width, const float* d,
                   const float* resid, float* out) {
  const size_t lds = (size_t)nout * width * sizeof(float);
  k_dense_t<<<grid_for((size_t)R * width), 256, lds, c.s>>>(R, W, nin, nout, koff, width, d, resid, out);
  HDG_CHECK_LAUNCH("k_dense_t");
  return HDG_OK;
}

hdg_status rowsum(const Ctx& c, int width, const float* t, float* out, bool acc, bool via_mirror, int mode) {
  k_rowsum<<<grid_for((size_t)c.nfc * width), 256, 0, c.s>>>((int)c.nfc, width, c.mesh->d_row_ptr,
                                                              via_mirror ? c.g->mirror : nullptr, t, out, acc ? 1 : 0,
                                                              mode, c.erow(), c.col(), c.ftype());
  HDG_CHECK_LAUNCH("k_rowsum");
  return HDG_OK;
}

hdg_status wgrad(const Ctx& c, int R, const Segs& in, const float* d, int nout, double* part, float* gW, float* gb) {
  const int P = nout * (in.nin + 1);
  k_wgrad_partial<<<::dim3(kWgChunks, (P + 255) / 256), 256, 0, c.s>>>(R, in, d, nout, part);
  k_wgrad_final<<<(P + 255) / 256, 256, 0, c.s>>>(nout, in.nin, part, gW, gb);
  HDG_CHECK_LAUNCH("k_wgrad");
  return HDG_OK;
}

Segs segs1(const float* a, const int* ga, int wa) {
  Segs s{};
  s.s[0] = {a, ga, wa};
  s.n = 1;
  s.nin = wa;
  return s;
}

Segs segs2(const float* a, const int* ga, int wa, const float* b, const int* gb, int wb) {
  Segs s{};
  s.s[0] = {a, ga, wa};
  s.s[1] = {b, gb, wb};
  s.n = 2;
  s.nin = wa + wb;
  return s;
}

Segs segs3(const float* a, const int* ga, int wa, const float* b, const int* gb, int wb, const float* cc,
           const int* gc, int wc) {
  Segs s{};
  s.s[0] = {a, ga, wa};
  s.s[1] = {b, gb, wb};
  s.s[2] = {cc, gc, wc};
  s.n = 3;
  s.nin = wa + wb + wc;
  return s;
}

#define GNN_TRY(x)              \
  do {                          \
    hdg_status st__ = (x);      \
    if (st__) return st__;      \
  } while (0)

hdg_status forward(const Ctx& c, const hdg_gnn_shape& s, const Layout& L, const float* th, Work& w, float* N,
                   float* Bp) {
  const int h = s.hidden, fe = s.d2 * s.d2, nfc = (int)c.nfc, nnzb = (int)c.nnzb;
  GNN_TRY(dense(c, nfc, segs1(c.g->node, nullptr, kF0), th + L.W0, th + L.c0, h, 1, nullptr, nullptr, nullptr,
                w.X[0], SEL_ALL));
  GNN_TRY(dense(c, nnzb, segs1(c.g->Hs, nullptr, fe), th + L.We, th + L.ce, h, 1, nullptr, nullptr, nullptr, w.Eh,
                SEL_OFF));
  for (int l = 0; l < s.layers; ++l) {
    GNN_TRY(dense(c, nnzb, segs3(w.X[l], c.erow(), h, w.X[l], c.col(), h, w.Eh, nullptr, h), th + L.Wm[l],
                  th + L.cm[l], h, 1, nullptr, nullptr, w.V[l], w.M, SEL_OFF));
    GNN_TRY(rowsum(c, h, w.M, w.Agg[l], false, false, SEL_OFF));
    GNN_TRY(dense(c, nfc, segs2(w.X[l], nullptr, h, w.Agg[l], nullptr, h), th + L.Wu[l], th + L.cu[l], h, 1, w.X[l],
                  nullptr, w.U[l], w.X[l + 1], SEL_ALL));
  }
  const int Lx = s.layers;
  GNN_TRY(dense(c, nnzb, segs3(w.X[Lx], c.erow(), h, w.X[Lx], c.col(), h, w.Eh, nullptr, h), th + L.Wo, th + L.co, fe,
                0, nullptr, c.g->Hs, nullptr, N, SEL_HEAD));
  k_mirror_upper<<<grid_for((size_t)nnzb * fe), 256, 0, c.s>>>(nnzb, s.d2, c.erow(), c.col(), c.g->mirror, N);
  const int fb = s.d2 * (s.d2 + 1) / 2;
  return dense(c, nfc, segs1(w.X[Lx], nullptr, h), th + L.Wb, th + L.cb, fb, 0, nullptr, nullptr, nullptr, Bp,
               SEL_FREE);
}

hdg_status backward(const Ctx& c, const hdg_gnn_shape& s, const Layout& L, const float* th, Work& w, float* gr) {
  const int h = s.hidden, fe = s.d2 * s.d2, nfc = (int)c.nfc, nnzb = (int)c.nnzb, Lx = s.layers;
  const int fb = s.d2 * (s.d2 + 1) / 2;
  // node head (w.dB is zero on Dirichlet faces)
  GNN_TRY(wgrad(c, nfc, segs1(w.X[Lx], nullptr, h), w.dB, fb, w.wpart, gr + L.Wb, gr + L.cb));
  GNN_TRY(dense_t(c, nfc, th + L.Wb, h, fb, 0, h, w.dB, nullptr, w.dX));
  // edge head
  GNN_TRY(wgrad(c, nnzb, segs3(w.X[Lx], c.erow(), h, w.X[Lx], c.col(), h, w.Eh, nullptr, h), w.dD, fe, w.wpart,
                gr + L.Wo, gr + L.co));
  GNN_TRY(dense_t(c, nnzb, th + L.Wo, 3 * h, fe, 0, h, w.dD, nullptr, w.t));
  GNN_TRY(rowsum(c, h, w.t, w.dX, true, false, SEL_HEAD));
  GNN_TRY(dense_t(c, nnzb, th + L.Wo, 3 * h, fe, h, h, w.dD, nullptr, w.t));
  GNN_TRY(rowsum(c, h, w.t, w.dX, true, true, SEL_HEAD));
  GNN_TRY(dense_t(c, nnzb, th + L.Wo, 3 * h, fe, 2 * h, h, w.dD, nullptr, w.dEh));
  for (int l = Lx - 1; l >= 0; --l) {
    // X_{l+1} = X_l + relu(U_l),  U_l = Wu [X_l; Agg_l] + cu
    k_relu_grad<<<grid_for((size_t)nfc * h), 256, 0, c.s>>>(nfc, h, w.dX, nullptr, w.U[l], w.M, SEL_ALL, c.erow(),
                                                             c.col(), c.ftype());
    GNN_TRY(wgrad(c, nfc, segs2(w.X[l], nullptr, h, w.Agg[l], nullptr, h), w.M, h, w.wpart, gr + L.Wu[l],
                  gr + L.cu[l]));
    GNN_TRY(dense_t(c, nfc, th + L.Wu[l], 2 * h, h, 0, h, w.M, w.dX, w.dXin));
    GNN_TRY(dense_t(c, nfc, th + L.Wu[l], 2 * h, h, h, h, w.M, nullptr, w.dX));  // dAgg (dX is free now)
    // M_e = relu(V_e), Agg_i = sum_e M_e  ->  dV_e = dAgg_{row(e)} (V_e > 0)
    k_relu_grad<<<grid_for((size_t)nnzb * h), 256, 0, c.s>>>(nnzb, h, w.dX, c.erow(), w.V[l], w.dV, SEL_OFF,
                                                              c.erow(), c.col(), c.ftype());
    GNN_TRY(wgrad(c, nnzb, segs3(w.X[l], c.erow(), h, w.X[l], c.col(), h, w.Eh, nullptr, h), w.dV, h, w.wpart,
                  gr + L.Wm[l], gr + L.cm[l]));
    GNN_TRY(dense_t(c, nnzb, th + L.Wm[l], 3 * h, h, 0, h, w.dV, nullptr, w.t));
    GNN_TRY(rowsum(c, h, w.t, w.dXin, true, false, SEL_OFF));
    GNN_TRY(dense_t(c, nnzb, th + L.Wm[l], 3 * h, h, h, h, w.dV, nullptr, w.t));
    GNN_TRY(rowsum(c, h, w.t, w.dXin, true, true, SEL_OFF));
    GNN_TRY(dense_t(c, nnzb, th + L.Wm[l], 3 * h, h, 2 * h, h, w.dV, w.dEh, w.dEh));
    std::swap(w.dX, w.dXin);
  }
  // E = relu(We b + ce): the stored E is zero exactly where the pre-activation was <= 0
  k_relu_grad<<<grid_for((size_t)nnzb * h), 256, 0, c.s>>>(nnzb, h, w.dEh, nullptr, w.Eh, w.dV, SEL_OFF, c.erow(),
                                                            c.col(), c.ftype());
  GNN_TRY(wgrad(c, nnzb, segs1(c.g->Hs, nullptr, fe), w.dV, h, w.wpart, gr + L.We, gr + L.ce));
  k_relu_grad<<<grid_for((size_t)nfc * h), 256, 0, c.s>>>(nfc, h, w.dX, nullptr, w.X[0], w.M, SEL_ALL, c.erow(),
                                                           c.col(), c.ftype());
  GNN_TRY(wgrad(c, nfc, segs1(c.g->node, nullptr, kF0), w.M, h, w.wpart, gr + L.W0, gr + L.c0));
  HDG_CHECK_LAUNCH("hdg_gnn backward");
  return HDG_OK;
}

hdg_status check_common(const hdg_gnn_shape* s, const hdg_mesh* mesh, const hdg_gnn_graph* g, const char* who) {
  GNN_TRY(check_shape(s, who));
  if (!mesh || !g || !g->Hs || !g->Linv || !g->node || !g->erow || !g->mirror || mesh->nfc < 1 ||
      !mesh->d_row_ptr || !mesh->d_col_idx || !mesh->d_ftype)
    return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": NULL argument or unexpanded mesh");
  return HDG_OK;
}

template <int D2>
hdg_status build_graph(const hdg_mesh* m, const double* H, const hdg_gnn_graph* g, double* Linv64, hipStream_t s) {
  const int nfc = (int)m->nfc, nnzb = (int)m->nnzb;
  k_erow<<<(nfc + 255) / 256, 256, 0, s>>>(nfc, m->d_row_ptr, g->erow);
  k_gnn_diag<D2><<<(nfc + 63) / 64, 64, 0, s>>>(nfc, m->d_diag, H, Linv64, g->Linv);
  k_gnn_edges<D2><<<(nnzb + 63) / 64, 64, 0, s>>>(nnzb, m->d_row_ptr, m->d_col_idx, g->erow, H, Linv64, g->Hs,
                                                  g->mirror);
  k_gnn_nodes<<<(nfc + 255) / 256, 256, 0, s>>>(nfc, D2 * D2, m->d_row_ptr, m->d_col_idx, m->d_ftype, m->d_area,
                                                std::pow((double)nfc, 2.0 / 3.0), g->Hs, g->node);
  HDG_CHECK_LAUNCH("hdg_gnn_build_graph");
  return HDG_OK;
}

}  // namespace

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who);

}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_gnn_param_count(const hdg_gnn_shape* shape, int64_t* n) {
  GNN_TRY(check_shape(shape, "hdg_gnn_param_count"));
  if (!n) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_param_count: n is NULL");
  *n = layout(*shape).total;
  return HDG_OK;
}

extern "C" hdg_status hdg_gnn_graph_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, size_t* bytes) {
  if (!disc || !mesh || !bytes) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_graph_workspace_size: NULL argument");
  *bytes = (size_t)mesh->nfc * disc->host.d2 * disc->host.d2 * sizeof(double);
  return HDG_OK;
}

extern "C" hdg_status hdg_gnn_build_graph(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_H,
                                          hdg_gnn_graph* graph, void* d_ws, size_t ws_bytes, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_gnn_build_graph");
  if (st) return st;
  if (!d_H || !graph || !graph->Hs || !graph->Linv || !graph->node || !graph->erow || !graph->mirror || !d_ws ||
      !mesh->d_area || !mesh->d_ftype)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_build_graph: NULL argument");
  const int d2 = disc->host.d2;
  if (ws_bytes < (size_t)mesh->nfc * d2 * d2 * sizeof(double))
    return set_error(HDG_ERR_WORKSPACE, "hdg_gnn_build_graph: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  double* L64 = (double*)d_ws;
  switch (d2) {
    case 1: return build_graph<1>(mesh, d_H, graph, L64, s);
    case 3: return build_graph<3>(mesh, d_H, graph, L64, s);
    case 6: return build_graph<6>(mesh, d_H, graph, L64, s);
    case 10: return build_graph<10>(mesh, d_H, graph, L64, s);
    case 15: return build_graph<15>(mesh, d_H, graph, L64, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_gnn_build_graph: unsupported block size");
}

extern "C" hdg_status hdg_gnn_workspace_size(const hdg_gnn_shape* shape, const hdg_mesh* mesh, int nprobe,
                                             size_t* bytes) {
  GNN_TRY(check_shape(shape, "hdg_gnn_workspace_size"));
  if (!mesh || !bytes || nprobe < 0) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_workspace_size: bad argument");
  *bytes = work_bytes(*shape, mesh->nfc, mesh->nnzb, nprobe, false, nullptr, nullptr, 0, nullptr);
  return HDG_OK;
}

extern "C" hdg_status hdg_gnn_forward(const hdg_gnn_shape* shape, const float* d_params, const hdg_mesh* mesh,
                                      const hdg_gnn_graph* graph, float* d_N, float* d_B, void* d_ws, size_t ws_bytes,
                                      void* stream) {
  GNN_TRY(check_common(shape, mesh, graph, "hdg_gnn_forward"));
  if (!d_params || !d_N || !d_B || !d_ws) return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_forward: NULL argument");
  Work w;
  bool ok = false;
  work_bytes(*shape, mesh->nfc, mesh->nnzb, 0, true, &w, d_ws, ws_bytes, &ok);
  if (!ok) return set_error(HDG_ERR_WORKSPACE, "hdg_gnn_forward: workspace too small");
  Ctx c{(hipStream_t)stream, mesh->nfc, mesh->nnzb, mesh, graph};
  return forward(c, *shape, layout(*shape), d_params, w, d_N, d_B);
}

extern "C" hdg_status hdg_gnn_loss_grad(const hdg_gnn_shape* shape, const float* d_params, const hdg_mesh* mesh,
                                        const hdg_gnn_graph* graph, const float* d_probes, int nprobe, float* d_N,
                                        float* d_B, double* d_loss, float* d_grad, void* d_ws, size_t ws_bytes,
                                        void* stream) {
  GNN_TRY(check_common(shape, mesh, graph, "hdg_gnn_loss_grad"));
  if (!d_params || !d_probes || nprobe < 1 || !d_N || !d_B || !d_loss || !d_ws)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_loss_grad: NULL argument or nprobe < 1");
  Work w;
  bool ok = false;
  work_bytes(*shape, mesh->nfc, mesh->nnzb, nprobe, true, &w, d_ws, ws_bytes, &ok);
  if (!ok) return set_error(HDG_ERR_WORKSPACE, "hdg_gnn_loss_grad: workspace too small");
  Ctx c{(hipStream_t)stream, mesh->nfc, mesh->nnzb, mesh, graph};
  const Layout L = layout(*shape);
  GNN_TRY(forward(c, *shape, L, d_params, w, d_N, d_B));
  const int d2 = shape->d2, nfc = (int)mesh->nfc;
  const size_t n = (size_t)nfc * d2;
  k_apply_BT<<<grid_for(n * nprobe), 256, 0, c.s>>>(nfc, d2, nprobe, d_B, d_probes, w.y);
  k_apply_GT<<<grid_for(n * nprobe), 256, 0, c.s>>>(nfc, d2, nprobe, mesh->d_row_ptr, mesh->d_col_idx, graph->mirror,
                                                     d_N, w.y, w.u);
  k_spmv_hs<<<grid_for(n * nprobe), 256, 0, c.s>>>(nfc, d2, nprobe, mesh->d_row_ptr, mesh->d_col_idx, graph->Hs, w.u,
                                                    w.hu);
  const double scale = 1.0 / ((double)nprobe * (double)n);
  k_dot_part<<<kRedB, kRedT, 0, c.s>>>(w.u, w.hu, n * nprobe, w.part);
  k_dot_fin<<<1, kRedT, 0, c.s>>>(w.part, scale, w.loss);  // T
  k_logdiag_part<<<kRedB, kRedT, 0, c.s>>>(nfc, d2, d_B, w.part);
  k_loss_fin<<<1, kRedT, 0, c.s>>>(w.part, w.loss, 2.0 / (double)n, d_loss);
  HDG_CHECK_LAUNCH("hdg_gnn_loss_grad loss");
  if (!d_grad) return HDG_OK;
  k_dN<<<grid_for((size_t)mesh->nnzb * d2 * d2), 256, 0, c.s>>>((int)mesh->nnzb, d2, nprobe, n, graph->erow,
                                                                  mesh->d_col_idx, mesh->d_ftype, w.y, w.hu, w.loss,
                                                                  2.0 * scale, w.dD);
  k_apply_G<<<grid_for(n * nprobe), 256, 0, c.s>>>(nfc, d2, nprobe, mesh->d_row_ptr, mesh->d_col_idx, d_N, w.hu, w.wv);
  k_dbeta<<<grid_for((size_t)nfc * d2 * (d2 + 1) / 2), 256, 0, c.s>>>(nfc, d2, nprobe, n, mesh->d_ftype, d_B, d_probes,
                                                                        w.wv, w.loss, 2.0 * scale, 2.0 / (double)n,
                                                                        w.dB);
  return backward(c, *shape, L, d_params, w, d_grad);
}

extern "C" hdg_status hdg_gnn_adam(int64_t n, float* d_params, const float* d_grad, float* d_m, float* d_v, int step,
                                   float lr, float beta1, float beta2, float eps, void* stream) {
  if (n < 1 || !d_params || !d_grad || !d_m || !d_v || step < 1)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_gnn_adam: bad argument");
  const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
  k_adam<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(n, d_params, d_grad, d_m, d_v, lr, beta1, beta2,
                                                                       eps, c1, c2);
  HDG_CHECK_LAUNCH("hdg_gnn_adam");
  return HDG_OK;
}
