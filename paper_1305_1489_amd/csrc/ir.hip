// Static condensation with FP32 local factorisations and FP64 iterative refinement
// (degrees 1..3).  The element blocks are those of Sections 3-4; the local solve and
// condensation follow eq 5.1-5.6.
//
// Local system (eq 5.1-5.4), with unknowns [q_x; q_y; q_z; u]:
//     A1 = [ M  .  .  -C_x^T ;  .  M  .  -C_y^T ;  .  .  M  -C_z^T ;  C_x C_y C_z  Mc + tauPP ]
//     B  = [A2 | Af]  (A2 = [n_x DP^T; n_y DP^T; n_z DP^T; -tauDP^T], Af = [0; 0; 0; f])
// X = A1^{-1} B is computed by iterative refinement:
//     X = 0;  repeat  R = B - A1 X (FP64),  X += P(R)
// until every right-hand-side column has settled: its correction is below 1e-15 of that
// column of X, or has stopped shrinking below 1e-12 of it (the rounding floor); a sweep
// limit marks the element as not converged.  P is the block
// elimination of A1 with FP32 factors:
//     Y_s = M^{-1} R_s,   U = S^{-1} (R_u - sum_s C_s Y_s),   Q_s = Y_s + M^{-1} C_s^T U,
//     S = Mc + tauPP + sum_s C_s M^{-1} C_s^T.
// M^{-1} and S^{-1} are formed in FP32 as Li^T Li from the FP32 Cholesky factor.  Every
// multi-column FP32 product (the inverse factors, S, and each application of P) runs on
// the matrix cores (v_mfma_f32_16x16x4f32), with operands staged in LDS and padded to
// multiples of 16.  The FP64 part is: the element blocks, the residual through the
// block-structured A1, the solution X, and
//     C^K = A3 X_2 + tauDD,   Cf^K = A3 X_f,   A3 = [n_x DP, n_y DP, n_z DP, tauDP]
// with the scatter of eq 6.5 (upper triangle mirrored, atomic adds onto zeros on the
// diagonal blocks and F, as in the FP64 kernels).  X is kept for the reconstruction:
//     [q; u] = X_f - X_2 uhat_K   (Section 6, "Reconstruction").
//
// One element per workgroup of four wavefronts; the GEMM tiles are dealt to the waves.
#include "device_common.h"

namespace hdg {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kIrThreads = 512;

__host__ __device__ constexpr int up16(int n) { return (n + 15) / 16 * 16; }

template <int K>
struct ID {
  static constexpr int D3 = dim3(K), D2 = dim2(K), M = 4 * D2, NR = M + 1, NQD = (K + 2) * (K + 2) * (K + 2);
  static constexpr int PD = up16(D3), PR = up16(NR), N4 = 4 * D3;
};

// C (Mr x Nc) = (acc ? C : 0) + sgn op(A) op(B), op(A) Mr x Kd, op(B) Kd x Nc, all in LDS,
// row-major with leading dimensions; Mr, Nc multiples of 16, Kd of 4.  Ends with a barrier.
__device__ void wg_gemm(int Mr, int Nc, int Kd, const float* A, int lda, bool ta, const float* B, int ldb, bool tb,
                        float* C, int ldc, bool acc, float sgn) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int tiles = (Mr / 16) * (Nc / 16);
  for (int t = wave; t < tiles; t += nw) {
    const int tm = t / (Nc / 16), tn = t % (Nc / 16);
    v4f d;
    if (acc) {
#pragma unroll
      for (int i = 0; i < 4; ++i) d[i] = C[(tm * 16 + 4 * k4 + i) * ldc + tn * 16 + r16];
    } else {
      d = v4f{0.f, 0.f, 0.f, 0.f};
    }
    for (int kk = 0; kk < Kd; kk += 4) {
      const int ar = tm * 16 + r16, ak = kk + k4;
      const float a = sgn * (ta ? A[ak * lda + ar] : A[ar * lda + ak]);
      const int bk = kk + k4, bc = tn * 16 + r16;
      const float b = tb ? B[bc * ldb + bk] : B[bk * ldb + bc];
      d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) C[(tm * 16 + 4 * k4 + i) * ldc + tn * 16 + r16] = d[i];
  }
  __syncthreads();
}

// Lower Cholesky factor of the n x n leading block of A (FP32, leading dimension ld, in
// place), then Li = L^{-1} (lower, ld) by column substitution; entries past n are left.
__device__ void chol_inv_f32(float* A, int ld, int n, float* Li) {
  const int t = threadIdx.x, nt = blockDim.x;
  for (int j = 0; j < n; ++j) {
    if (t == 0) {
      float s = A[j * ld + j];
      for (int k = 0; k < j; ++k) s -= A[j * ld + k] * A[j * ld + k];
      A[j * ld + j] = sqrtf(s);
    }
    __syncthreads();
    const float inv = 1.0f / A[j * ld + j];
    for (int i = j + 1 + t; i < n; i += nt) {
      float s = A[i * ld + j];
      for (int k = 0; k < j; ++k) s -= A[i * ld + k] * A[j * ld + k];
      A[i * ld + j] = s * inv;
    }
    __syncthreads();
  }
  for (int c = t; c < n; c += nt) {  // column c of L^{-1}
    for (int i = 0; i < n; ++i) {
      float s = (i == c) ? 1.0f : 0.0f;
      for (int k = c; k < i; ++k) s -= A[i * ld + k] * Li[k * ld + c];
      Li[i * ld + c] = (i < c) ? 0.0f : s / A[i * ld + i];
    }
  }
  __syncthreads();
}

template <int K>
struct IrSmem {
  using D = ID<K>;
  static constexpr int PD = D::PD, PR = D::PR, D3 = D::D3, NR = D::NR, N4 = D::N4, NQD = D::NQD;
  // FP64
  double wk[NQD], wc[NQD], wf[NQD];
  double M[D3 * D3], Sd[D3 * D3], Cs[3][D3 * D3], f[D3];
  double X[N4 * NR];
  int flag;
  double dprev[D::NR];  // each column's previous correction size
  // FP32, padded
  float Minv[PD * PD], Sinv[PD * PD], Wk[PD * PR], C32[3][PD * PD], G[3][PD * PD];
  float R[3][PD * PR], Ru[PD * PR], Y[3][PD * PR];
};

template <int K>
__global__ void __launch_bounds__(kIrThreads) k_condense_ir(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                            const double* __restrict__ cco,
                                                            const double* __restrict__ fco,
                                                            const double* __restrict__ tau, double* __restrict__ H,
                                                            double* __restrict__ F, double* __restrict__ Xout,
                                                            int max_sweeps, int* __restrict__ sweeps_out,
                                                            const int* __restrict__ elems, int nwork,
                                                            double* __restrict__ Cout, double* __restrict__ Cfout) {
  using D = ID<K>;
  constexpr int D3 = D::D3, D2 = D::D2, M = D::M, NR = D::NR, NQD = D::NQD, PD = D::PD, PR = D::PR, N4 = D::N4;
  __shared__ IrSmem<K> sm;
  __shared__ ElemGeom sg;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int E = elems ? elems[w] : w;
    if (E < 0 || E >= mesh.nelt) continue;  // uniform across the workgroup
    __syncthreads();
    if (t == 0) load_geometry(E, mesh, tau, sg);
    // zero the padded FP32 buffers (their padding must stay zero / identity)
    for (int i = t; i < PD * PR; i += nt) {
      sm.Ru[i] = 0.f;
      sm.Wk[i] = 0.f;
      for (int s = 0; s < 3; ++s) sm.R[s][i] = 0.f;
    }
    for (int i = t; i < PD * PD; i += nt)
      for (int s = 0; s < 3; ++s) sm.C32[s][i] = 0.f;
    for (int i = t; i < N4 * NR; i += nt) sm.X[i] = 0.0;
    __syncthreads();
    const ElemGeom& g = sg;
    for (int q = t; q < NQD; q += nt) {
      const double wq = g.vol * tb.vol_w[q];
      sm.wk[q] = wq / kappa[(size_t)E * NQD + q];
      sm.wc[q] = wq * cco[(size_t)E * NQD + q];
      sm.wf[q] = wq * fco[(size_t)E * NQD + q];
    }
    __syncthreads();
    // ---- FP64 element blocks
    for (int idx = t; idx < D3 * D3; idx += nt) {
      const int i = idx / D3, j = idx % D3;
      double sk = 0, sc = 0;
      for (int q = 0; q < NQD; ++q) {
        const double pp = tb.P[q * D3 + i] * tb.P[q * D3 + j];
        sk += sm.wk[q] * pp;
        sc += sm.wc[q] * pp;
      }
      for (int l = 0; l < 4; ++l) sc += g.T[l] * tb.PP[(l * D3 + i) * D3 + j];
      sm.M[idx] = sk;
      sm.Sd[idx] = sc;
      for (int s = 0; s < 3; ++s) {
        double v = 0;
        for (int h = 0; h < 3; ++h) v += g.a[s][h] * tb.Chat[(h * D3 + i) * D3 + j];
        sm.Cs[s][idx] = v;
        sm.C32[s][i * PD + j] = (float)v;
      }
    }
    for (int i = t; i < D3; i += nt) {
      double s = 0;
      for (int q = 0; q < NQD; ++q) s += sm.wf[q] * tb.P[q * D3 + i];
      sm.f[i] = s;
    }
    __syncthreads();
    // FP32 copy of M padded with the identity (in Wk as scratch)
    for (int idx = t; idx < PD * PD; idx += nt) {
      const int i = idx / PD, j = idx % PD;
      sm.Wk[idx] = (i < D3 && j < D3) ? (float)sm.M[i * D3 + j] : (i == j ? 1.f : 0.f);
    }
    __syncthreads();
    // ---- FP32 factors: M^{-1} = Li^T Li
    chol_inv_f32(sm.Wk, PD, PD, sm.Sinv);
    wg_gemm(PD, PD, PD, sm.Sinv, PD, true, sm.Sinv, PD, false, sm.Minv, PD, false, 1.f);
    // G_s = M^{-1} C_s^T
    for (int s = 0; s < 3; ++s) wg_gemm(PD, PD, PD, sm.Minv, PD, false, sm.C32[s], PD, true, sm.G[s], PD, false, 1.f);
    // S = Mc + tauPP + sum_s C_s G_s, then S^{-1} = Li^T Li
    for (int idx = t; idx < PD * PD; idx += nt) {
      const int i = idx / PD, j = idx % PD;
      sm.Wk[idx] = (i < D3 && j < D3) ? (float)sm.Sd[i * D3 + j] : (i == j ? 1.f : 0.f);
    }
    __syncthreads();
    for (int s = 0; s < 3; ++s) wg_gemm(PD, PD, PD, sm.C32[s], PD, false, sm.G[s], PD, false, sm.Wk, PD, true, 1.f);
    chol_inv_f32(sm.Wk, PD, PD, sm.Y[0]);
    wg_gemm(PD, PD, PD, sm.Y[0], PD, true, sm.Y[0], PD, false, sm.Sinv, PD, false, 1.f);
    for (int i = t; i < PD * PR; i += nt)
      for (int s = 0; s < 3; ++s) sm.Y[s][i] = 0.f;
    __syncthreads();

    // ---- iterative refinement
    int sweep = 0;
    bool converged = false;
    for (; sweep < max_sweeps; ++sweep) {
      // R = B - A1 X (FP64), stored as FP32
      for (int idx = t; idx < N4 * NR; idx += nt) {
        const int row = idx / NR, c = idx % NR, blk = row / D3, j = row % D3;
        double b = 0;
        if (c < M) {
          const int l = c / D2, ii = c % D2;
          const double dp = tb.DP[((g.mu[l] * 4 + l) * D2 + ii) * D3 + j];
          b = blk < 3 ? g.n[l][blk] * dp : -g.T[l] * dp;
        } else if (blk == 3) {
          b = sm.f[j];
        }
        double ax = 0;
        if (blk < 3) {  // M X_s - C_s^T X_u
          for (int k = 0; k < D3; ++k)
            ax += sm.M[j * D3 + k] * sm.X[(blk * D3 + k) * NR + c] - sm.Cs[blk][k * D3 + j] * sm.X[(3 * D3 + k) * NR + c];
        } else {        // sum_s C_s X_s + (Mc + tauPP) X_u
          for (int k = 0; k < D3; ++k) {
            ax += sm.Sd[j * D3 + k] * sm.X[(3 * D3 + k) * NR + c];
            for (int s = 0; s < 3; ++s) ax += sm.Cs[s][j * D3 + k] * sm.X[(s * D3 + k) * NR + c];
          }
        }
        const float rv = (float)(b - ax);
        if (blk < 3)
          sm.R[blk][j * PR + c] = rv;
        else
          sm.Ru[j * PR + c] = rv;
      }
      __syncthreads();
      // P(R): Y_s = M^{-1} R_s;  Ru -= sum_s C_s Y_s;  U = S^{-1} Ru (in Wk);  Y_s += G_s U
      for (int s = 0; s < 3; ++s) wg_gemm(PD, PR, PD, sm.Minv, PD, false, sm.R[s], PR, false, sm.Y[s], PR, false, 1.f);
      for (int s = 0; s < 3; ++s) wg_gemm(PD, PR, PD, sm.C32[s], PD, false, sm.Y[s], PR, false, sm.Ru, PR, true, -1.f);
      wg_gemm(PD, PR, PD, sm.Sinv, PD, false, sm.Ru, PR, false, sm.Wk, PR, false, 1.f);
      for (int s = 0; s < 3; ++s) wg_gemm(PD, PR, PD, sm.G[s], PD, false, sm.Wk, PR, false, sm.Y[s], PR, true, 1.f);
      // X += [Y; U], and per right-hand-side column the size of the correction against the
      // size of that column of X (one thread per column).  A column is settled once its
      // correction is at most 1e-15 of its own scale, or once the correction stops shrinking
      // (at least half the previous one) at a level already below 1e-12: the FP64 residual's
      // rounding floor, about cond(A1) eps, which further sweeps cannot go below.  Every
      // column is judged on its own scale, so a small column (f, or one face's columns) is
      // refined as far as the large ones.
      if (t == 0) sm.flag = 0;
      __syncthreads();
      for (int c = t; c < NR; c += nt) {
        double dmax = 0, xmax = 0;
        for (int row = 0; row < N4; ++row) {
          const int blk = row / D3, j = row % D3, idx = row * NR + c;
          const double dv = blk < 3 ? (double)sm.Y[blk][j * PR + c] : (double)sm.Wk[j * PR + c];
          const double xv = sm.X[idx] + dv;
          sm.X[idx] = xv;
          dmax = fmax(dmax, fabs(dv));
          xmax = fmax(xmax, fabs(xv));
        }
        const bool small = !(dmax > 1e-15 * xmax);
        const bool floor_reached = sweep > 0 && dmax >= 0.5 * sm.dprev[c] && !(dmax > 1e-12 * xmax);
        if (!small && !floor_reached) sm.flag = 1;  // every writer stores the same value
        sm.dprev[c] = dmax;
      }
      __syncthreads();
      const bool more = sm.flag != 0;
      __syncthreads();
      if (!more) {
        converged = true;
        ++sweep;
        break;
      }
    }
    // max_sweeps + 1 marks an element whose last correction still exceeded the bound
    if (sweeps_out && t == 0) sweeps_out[w] = converged ? sweep : max_sweeps + 1;
    // ---- C^K = A3 X_2 + tauDD (upper triangle, mirrored), Cf^K = A3 X_f; scatter
    for (int idx = t; idx < M * NR; idx += nt) {
      const int a = idx / NR, b = idx % NR;
      if (b < M && b < a) continue;
      const int la = a / D2, ia = a % D2;
      const double* dpa = tb.DP + ((g.mu[la] * 4 + la) * D2 + ia) * D3;
      double v = 0;
      for (int j = 0; j < D3; ++j) {
        const double dp = dpa[j];
        v += dp * (g.n[la][0] * sm.X[j * NR + b] + g.n[la][1] * sm.X[(D3 + j) * NR + b] +
                   g.n[la][2] * sm.X[(2 * D3 + j) * NR + b] + g.T[la] * sm.X[(3 * D3 + j) * NR + b]);
      }
      if (b == M) {
        if (Cfout)
          Cfout[(size_t)w * M + a] = v;
        else
          unsafeAtomicAdd(&F[(size_t)mesh.d_facebyele[4 * E + la] * D2 + ia], v);
        continue;
      }
      if (a == b) v += g.T[la];
      if (Cout) {
        Cout[((size_t)w * M + a) * M + b] = v;
        Cout[((size_t)w * M + b) * M + a] = v;
        continue;
      }
      const int lb = b / D2, ib = b % D2;
      const size_t s1 = mesh.d_slot[16 * E + 4 * la + lb];
      if (la == lb) {
        unsafeAtomicAdd(&H[(s1 * D2 + ia) * D2 + ib], v);
        if (ia != ib) unsafeAtomicAdd(&H[(s1 * D2 + ib) * D2 + ia], v);
      } else {
        const size_t s2 = mesh.d_slot[16 * E + 4 * lb + la];
        H[(s1 * D2 + ia) * D2 + ib] = v;
        H[(s2 * D2 + ib) * D2 + ia] = v;
      }
    }
    if (Xout)
      for (int idx = t; idx < N4 * NR; idx += nt) Xout[(size_t)w * N4 * NR + idx] = sm.X[idx];
  }
}

template <int D2>
__global__ void k_zero_diag_ir(const int* __restrict__ diag, int nfc, double* __restrict__ H, double* __restrict__ F) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)nfc * D2 * D2) return;
  const size_t f = i / (D2 * D2), e = i % (D2 * D2);
  H[(size_t)diag[f] * D2 * D2 + e] = 0.0;
  if (e < D2) F[f * D2 + e] = 0.0;
}

// [q; u] = X_f - X_2 uhat_K, one thread per row of X
template <int K>
__global__ void k_recover_x(hdg_mesh mesh, const double* __restrict__ X, const double* __restrict__ uhat,
                            double* __restrict__ q, double* __restrict__ u) {
  using D = ID<K>;
  constexpr int D3 = D::D3, D2 = D::D2, M = D::M, NR = D::NR, N4 = D::N4;
  const size_t total = (size_t)mesh.nelt * N4;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const size_t E = idx / N4;
    const int row = (int)(idx % N4);
    const double* xr = X + (E * N4 + row) * NR;
    double v = xr[M];
    for (int l = 0; l < 4; ++l) {
      const double* uh = uhat + (size_t)mesh.d_facebyele[4 * E + l] * D2;
      for (int i = 0; i < D2; ++i) v -= xr[l * D2 + i] * uh[i];
    }
    if (row < 3 * D3)
      q[E * 3 * D3 + row] = v;
    else
      u[E * D3 + row - 3 * D3] = v;
  }
}

template <int K>
hdg_status run_ir(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c, const double* f,
                  const double* tau, double* H, double* F, double* X, int max_sweeps, int* sweeps, const int* elems,
                  int64_t n, double* Cout, double* Cfout, hipStream_t s) {
  using D = ID<K>;
  if (!Cout) {
    const size_t tot = (size_t)mesh->nfc * D::D2 * D::D2;
    k_zero_diag_ir<D::D2><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(mesh->d_diag, (int)mesh->nfc, H, F);
  }
  if (n == 0) return HDG_OK;
  const int grid = (int)std::min<int64_t>(n, 4 * device_cu_count());
  k_condense_ir<K><<<grid, kIrThreads, 0, s>>>(*mesh, disc->dev, kappa, c, f, tau, H, F, X, max_sweeps, sweeps, elems,
                                               (int)n, Cout, Cfout);
  HDG_CHECK_LAUNCH("k_condense_ir");
  return HDG_OK;
}

template <int K>
hdg_status run_recover_x(const hdg_mesh* mesh, const double* X, const double* uhat, double* q, double* u,
                         hipStream_t s) {
  const size_t tot = (size_t)mesh->nelt * ID<K>::N4;
  k_recover_x<K><<<(unsigned)std::min<size_t>((tot + 255) / 256, 65535), 256, 0, s>>>(*mesh, X, uhat, q, u);
  HDG_CHECK_LAUNCH("k_recover_x");
  return HDG_OK;
}

}  // namespace

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who);

}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_ir_store_len(const hdg_disc* disc, int64_t* n) {
  if (!disc || !n) return set_error(HDG_ERR_INVALID_ARG, "hdg_ir_store_len: NULL argument");
  const int d3 = disc->host.d3, m = 4 * disc->host.d2;
  *n = (int64_t)4 * d3 * (m + 1);
  return HDG_OK;
}

extern "C" hdg_status hdg_assemble_condense_ir(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                               const double* d_c, const double* d_f, const double* d_tau, double* d_H,
                                               double* d_F, double* d_X, int max_sweeps, int32_t* d_sweeps,
                                               void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_assemble_condense_ir");
  if (st) return st;
  if (!d_kappa || !d_c || !d_f || !d_tau || !d_H || !d_F || max_sweeps < 1 || max_sweeps > 20)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_assemble_condense_ir: NULL array or max_sweeps outside 1..20");
  hipStream_t s = (hipStream_t)stream;
  st = check_not_singular(disc, mesh, d_c, s, "hdg_assemble_condense_ir");
  if (st) return st;
  const int64_t n = mesh->nelt;
  switch (disc->host.k) {
    case 1: return run_ir<1>(disc, mesh, d_kappa, d_c, d_f, d_tau, d_H, d_F, d_X, max_sweeps, d_sweeps, nullptr, n, nullptr, nullptr, s);
    case 2: return run_ir<2>(disc, mesh, d_kappa, d_c, d_f, d_tau, d_H, d_F, d_X, max_sweeps, d_sweeps, nullptr, n, nullptr, nullptr, s);
    case 3: return run_ir<3>(disc, mesh, d_kappa, d_c, d_f, d_tau, d_H, d_F, d_X, max_sweeps, d_sweeps, nullptr, n, nullptr, nullptr, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_assemble_condense_ir: degrees 1..3 only");
}

extern "C" hdg_status hdg_export_local_ir(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                          const double* d_c, const double* d_f, const double* d_tau,
                                          const int32_t* d_elems, int64_t n, double* d_C, double* d_Cf,
                                          double* d_X, int max_sweeps, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_export_local_ir");
  if (st) return st;
  if (!d_kappa || !d_c || !d_f || !d_tau || !d_elems || !d_C || !d_Cf || n < 0 || max_sweeps < 1 || max_sweeps > 20)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_export_local_ir: NULL array, n < 0 or max_sweeps outside 1..20");
  hipStream_t s = (hipStream_t)stream;
  switch (disc->host.k) {
    case 1: return run_ir<1>(disc, mesh, d_kappa, d_c, d_f, d_tau, nullptr, nullptr, d_X, max_sweeps, nullptr, d_elems, n, d_C, d_Cf, s);
    case 2: return run_ir<2>(disc, mesh, d_kappa, d_c, d_f, d_tau, nullptr, nullptr, d_X, max_sweeps, nullptr, d_elems, n, d_C, d_Cf, s);
    case 3: return run_ir<3>(disc, mesh, d_kappa, d_c, d_f, d_tau, nullptr, nullptr, d_X, max_sweeps, nullptr, d_elems, n, d_C, d_Cf, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_export_local_ir: degrees 1..3 only");
}

extern "C" hdg_status hdg_recover_ir(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_X,
                                     const double* d_uhat, double* d_q, double* d_u, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_recover_ir");
  if (st) return st;
  if (!d_X || !d_uhat || !d_q || !d_u) return set_error(HDG_ERR_INVALID_ARG, "hdg_recover_ir: NULL array");
  hipStream_t s = (hipStream_t)stream;
  switch (disc->host.k) {
    case 0: return run_recover_x<0>(mesh, d_X, d_uhat, d_q, d_u, s);
    case 1: return run_recover_x<1>(mesh, d_X, d_uhat, d_q, d_u, s);
    case 2: return run_recover_x<2>(mesh, d_X, d_uhat, d_q, d_u, s);
    case 3: return run_recover_x<3>(mesh, d_X, d_uhat, d_q, d_u, s);
    case 4: return run_recover_x<4>(mesh, d_X, d_uhat, d_q, d_u, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_recover_ir: unsupported degree");
}
