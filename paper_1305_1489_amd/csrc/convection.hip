// Static condensation of the HDG method for convection-diffusion (Section 9, "Matrices for
// convection-diffusion problems"), degrees 0..3, FP64.
//
// The problem is  kappa^{-1} q + grad u = 0,  div(q + beta u) + c u = f,  with the numerical
// total flux  q.nu + (beta.nu) uhat + tau (u - uhat)  on the element boundaries.  Against the
// diffusion element of Sections 3-5 it adds
//   - to the u block of A1:   - sum_s E_s^T,  E_s[i][j] = int_K beta_s P_i d_s P_j   (eq 9.1)
//   - to the u rows of A2:    + (beta.n DP_l)^T,  (beta.n DP_l)[i][j] = int_{e_l} (beta.nu) D_i P_j
//   - to C^K:                 - beta.n DD_l on the diagonal blocks,
//                             (beta.n DD_l)[i][j] = int_{e_l} (beta.nu) D_i D_j,
// with A3 unchanged.  The beta integrals are quadrature sums: over the volume points
// (beta at hdg_qp_coords), and over the element's own points of each face, phi_l^K(qhat_r)
// (beta at hdg_elem_face_qp_coords), where the face basis of the global face is D(F_mu(qhat_r))
// with mu = perm(K, l) - 1 (eq 2.2).
//
// The local solve eliminates q through the Cholesky factor L of M = M_{1/kappa}:
//   G_s = L^{-1} C_s^T,   S = Mc + tauPP - sum_s E_s^T + sum_s G_s^T G_s,
//   Z_s = L^{-1} b_s,     u = S^{-1} (b_u - sum_s G_s^T Z_s),   q_s = L^{-T} (Z_s + G_s u),
// for every right-hand side [b_x; b_y; b_z; b_u] of B = [A2 | Af].  S is not symmetric; its
// symmetric part is that of M_{c + div(beta)/2} + sum_s G_s^T G_s plus the face terms
// (tau - beta.nu / 2) PP, positive definite when tau >= beta.nu / 2, so S is factored by LU
// without pivoting.  X = A1^{-1} B is kept for the reconstruction ([q; u] = X_f - X_2 uhat_K,
// hdg_recover_ir), and
//   C^K = A3 X_2 + tauDD - beta.n DD,   Cf^K = A3 X_f
// are scattered into H and F: every entry of C^K (H is not symmetric), off-diagonal blocks by
// their single writer, diagonal blocks and F by atomic adds onto zeros (two addends: the same
// bits in either order).
//
// One element per workgroup of four wavefronts, everything in LDS (78 KB at k = 3: two
// workgroups per CU); the factorisations and triangular solves update all rows of all
// right-hand sides in parallel at each elimination step.
#include "device_common.h"

namespace hdg {
namespace {

constexpr int kCdThreads = 256;

template <int K>
struct CdDims {
  static constexpr int D3 = dim3(K), D2 = dim2(K), M = 4 * D2, NR = M + 1, N4 = 4 * D3;
  static constexpr int NQD = (K + 2) * (K + 2) * (K + 2), NQD2 = (K + 2) * (K + 2);
};

template <int K>
struct CdSmem {
  using D = CdDims<K>;
  static constexpr int D3 = D::D3, D2 = D::D2, NR = D::NR, N4 = D::N4, NQD = D::NQD, NQD2 = D::NQD2;
  double wk[NQD], wc[NQD], wf[NQD];  // |K| w_q / kappa, |K| w_q c, |K| w_q f
  double gam[3][NQD];                // (w_q / 6) sum_s beta_s(x_q) a_{s h}
  double al[4][NQD2];                // w_r beta(x_r) . n_l  (|n_l| = |e_l|)
  double Mm[D3 * D3];                // M_{1/kappa}, then its Cholesky factor (lower)
  double S[D3 * D3];                 // the u Schur complement, then its LU factors
  double G[3][D3 * D3];              // C_s^T, then G_s = L^{-1} C_s^T
  double f[D3];
  double bnDP[4][D2 * D3];
  double bnDD[4][D2 * D2];
  double T[NQD * D3];                // T[q][i] = sum_h gam_h(q) dhat_h P_i(q)
  double X[N4 * NR];                 // [q_x; q_y; q_z; u] for every right-hand side; while the
                                     // element blocks are formed, the basis table P[q][i]
};
static_assert(CdDims<3>::NQD * CdDims<3>::D3 <= CdDims<3>::N4 * CdDims<3>::NR, "P staged in X");
// two workgroups per CU (160 KB of LDS)
static_assert(sizeof(CdSmem<3>) + sizeof(ElemGeom) <= 80 * 1024, "convection-diffusion LDS budget");

// In-place LU factorisation without pivoting (unit lower factor below the diagonal), all
// threads of the block, one (row, column) entry of the trailing block per thread and
// step; ends with a barrier.
template <int N>
__device__ void lds_lu_nopiv(double* A) {
  for (int p = 0; p < N; ++p) {
    const double inv = 1.0 / A[p * N + p];
    const int m = N - 1 - p;
    for (int e = threadIdx.x; e < m * (m + 1); e += blockDim.x) {  // column p + e % (m + 1)
      const int i = p + 1 + e / (m + 1), jj = e % (m + 1);
      if (jj == 0) continue;
      const int j = p + jj;
      A[i * N + j] -= (A[i * N + p] * inv) * A[p * N + j];
    }
    __syncthreads();
    for (int i = p + 1 + threadIdx.x; i < N; i += blockDim.x) A[i * N + p] *= inv;
    __syncthreads();
  }
}

// Triangular solves on NM sets of NC right-hand sides: set m holds its row r at
// X + m * mstride + r * ldx.  Column-oriented, so that each step updates all remaining rows
// of every right-hand side in parallel, with the operation order of row substitution
// (subtractions in increasing k, then the division).  L is row-major with leading
// dimension N; each ends with a barrier.
//   lds_forward_par<UNIT>:    X <- L^{-1} X  (UNIT: L has a unit diagonal, not stored)
//   lds_backward_par<TRANS>:  X <- L^{-T} X  (TRANS, L lower) or U^{-1} X (U upper)
template <int N, bool UNIT>
__device__ void lds_forward_par(const double* L, double* X, int ldx, int nc, int nm, int mstride) {
  for (int k = 0; k < N; ++k) {
    if (!UNIT) {
      for (int e = threadIdx.x; e < nm * nc; e += blockDim.x)
        X[(e / nc) * mstride + k * ldx + e % nc] /= L[k * N + k];
      __syncthreads();
    }
    const int rows = N - 1 - k, per = rows * nc;
    for (int e = threadIdx.x; e < nm * per; e += blockDim.x) {
      const int m = e / per, rc = e % per, r = k + 1 + rc / nc, c = rc % nc;
      double* x = X + m * mstride;
      x[r * ldx + c] -= L[r * N + k] * x[k * ldx + c];
    }
    __syncthreads();
  }
}

template <int N, bool TRANS>
__device__ void lds_backward_par(const double* L, double* X, int ldx, int nc, int nm, int mstride) {
  for (int k = N - 1; k >= 0; --k) {
    for (int e = threadIdx.x; e < nm * nc; e += blockDim.x)
      X[(e / nc) * mstride + k * ldx + e % nc] /= L[k * N + k];
    __syncthreads();
    const int per = k * nc;
    for (int e = threadIdx.x; e < nm * per; e += blockDim.x) {
      const int m = e / per, rc = e % per, r = rc / nc, c = rc % nc;
      double* x = X + m * mstride;
      x[r * ldx + c] -= (TRANS ? L[k * N + r] : L[r * N + k]) * x[k * ldx + c];
    }
    __syncthreads();
  }
}

template <int K>
__global__ void __launch_bounds__(kCdThreads) k_condense_cd(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                            const double* __restrict__ cco,
                                                            const double* __restrict__ fco,
                                                            const double* __restrict__ bvol,
                                                            const double* __restrict__ bface,
                                                            const double* __restrict__ tau, double* __restrict__ H,
                                                            double* __restrict__ F, double* __restrict__ Xout,
                                                            const int* __restrict__ elems, int nwork,
                                                            double* __restrict__ Cout, double* __restrict__ Cfout) {
  using D = CdDims<K>;
  constexpr int D3 = D::D3, D2 = D::D2, M = D::M, NR = D::NR, N4 = D::N4, NQD = D::NQD, NQD2 = D::NQD2;
  __shared__ CdSmem<K> sm;
  __shared__ ElemGeom sg;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int E = elems ? elems[w] : w;
    if (E < 0 || E >= mesh.nelt) continue;  // uniform across the workgroup
    __syncthreads();
    if (t == 0) load_geometry(E, mesh, tau, sg);
    __syncthreads();
    const ElemGeom& g = sg;
    for (int q = t; q < NQD; q += nt) {
      const size_t e = (size_t)E * NQD + q;
      const double wq = g.vol * tb.vol_w[q];
      sm.wk[q] = wq / kappa[e];
      sm.wc[q] = wq * cco[e];
      sm.wf[q] = wq * fco[e];
      const double w6 = tb.vol_w[q] / 6.0;
      const double b0 = bvol[3 * e], b1 = bvol[3 * e + 1], b2 = bvol[3 * e + 2];
      for (int h = 0; h < 3; ++h) sm.gam[h][q] = w6 * (b0 * g.a[0][h] + b1 * g.a[1][h] + b2 * g.a[2][h]);
    }
    for (int lr = t; lr < 4 * NQD2; lr += nt) {
      const int l = lr / NQD2, r = lr % NQD2;
      const double* b = bface + ((size_t)E * 4 * NQD2 + lr) * 3;
      sm.al[l][r] = tb.tri_w[r] * (b[0] * g.n[l][0] + b[1] * g.n[l][1] + b[2] * g.n[l][2]);
    }
    __syncthreads();
    // ---- element blocks: the basis table goes to LDS (in X, free until the right-hand
    // sides) and the beta-weighted reference gradients to T
    for (int idx = t; idx < NQD * D3; idx += nt) {
      const int q = idx / D3, i = idx % D3;
      sm.X[idx] = tb.P[idx];
      sm.T[idx] = sm.gam[0][q] * tb.Pg[q * D3 + i] + sm.gam[1][q] * tb.Pg[(NQD + q) * D3 + i] +
                  sm.gam[2][q] * tb.Pg[(2 * NQD + q) * D3 + i];
    }
    __syncthreads();
    for (int idx = t; idx < D3 * D3; idx += nt) {
      const int i = idx / D3, j = idx % D3;
      double sk = 0, sc = 0, se = 0;
      for (int q = 0; q < NQD; ++q) {
        const double pi = sm.X[q * D3 + i], pj = sm.X[q * D3 + j];
        sk += sm.wk[q] * pi * pj;
        sc += sm.wc[q] * pi * pj;
        se += pj * sm.T[q * D3 + i];  // (sum_s E_s^T)[i][j] = sum_q P_j sum_h gam_h grad_h P_i
      }
      for (int l = 0; l < 4; ++l) sc += g.T[l] * tb.PP[(l * D3 + i) * D3 + j];
      sm.Mm[idx] = sk;
      sm.S[idx] = sc - se;
      for (int s = 0; s < 3; ++s) {  // C_s^T[i][j] = C_s[j][i]
        double v = 0;
        for (int h = 0; h < 3; ++h) v += g.a[s][h] * tb.Chat[(h * D3 + j) * D3 + i];
        sm.G[s][idx] = v;
      }
    }
    for (int i = t; i < D3; i += nt) {
      double s = 0;
      for (int q = 0; q < NQD; ++q) s += sm.wf[q] * sm.X[q * D3 + i];
      sm.f[i] = s;
    }
    for (int idx = t; idx < 4 * D2 * D3; idx += nt) {
      const int l = idx / (D2 * D3), i = (idx / D3) % D2, j = idx % D3;
      const double* dm = tb.Dmu + (size_t)g.mu[l] * NQD2 * D2;
      const double* pf = tb.Pface + (size_t)l * NQD2 * D3;
      double s = 0;
      for (int r = 0; r < NQD2; ++r) s += sm.al[l][r] * dm[r * D2 + i] * pf[r * D3 + j];
      sm.bnDP[l][i * D3 + j] = s;
    }
    for (int idx = t; idx < 4 * D2 * D2; idx += nt) {
      const int l = idx / (D2 * D2), i = (idx / D2) % D2, j = idx % D2;
      const double* dm = tb.Dmu + (size_t)g.mu[l] * NQD2 * D2;
      double s = 0;
      for (int r = 0; r < NQD2; ++r) s += sm.al[l][r] * dm[r * D2 + i] * dm[r * D2 + j];
      sm.bnDD[l][i * D2 + j] = s;
    }
    __syncthreads();
    // ---- M = L L^T;  G_s = L^{-1} C_s^T;  S += sum_s G_s^T G_s;  S = LU
    lds_cholesky<D3>(sm.Mm, D3);
    lds_forward_par<D3, false>(sm.Mm, &sm.G[0][0], D3, D3, 3, D3 * D3);
    for (int idx = t; idx < D3 * D3; idx += nt) {
      const int i = idx / D3, j = idx % D3;
      double v = sm.S[idx];
      for (int s = 0; s < 3; ++s)
        for (int k = 0; k < D3; ++k) v += sm.G[s][k * D3 + i] * sm.G[s][k * D3 + j];
      sm.S[idx] = v;
    }
    // ---- right-hand sides B = [A2 | Af]
    for (int idx = t; idx < N4 * NR; idx += nt) {
      const int row = idx / NR, c = idx % NR, blk = row / D3, j = row % D3;
      double b = 0;
      if (c < M) {
        const int l = c / D2, ii = c % D2;
        const double dp = tb.DP[((g.mu[l] * 4 + l) * D2 + ii) * D3 + j];
        b = blk < 3 ? g.n[l][blk] * dp : -g.T[l] * dp + sm.bnDP[l][ii * D3 + j];
      } else if (blk == 3) {
        b = sm.f[j];
      }
      sm.X[idx] = b;
    }
    __syncthreads();
    lds_lu_nopiv<D3>(sm.S);
    // Z_s = L^{-1} b_s (in the q rows of X)
    lds_forward_par<D3, false>(sm.Mm, sm.X, NR, NR, 3, D3 * NR);
    // b_u -= sum_s G_s^T Z_s
    for (int idx = t; idx < D3 * NR; idx += nt) {
      const int j = idx / NR, c = idx % NR;
      double v = sm.X[(3 * D3 + j) * NR + c];
      for (int s = 0; s < 3; ++s)
        for (int k = 0; k < D3; ++k) v -= sm.G[s][k * D3 + j] * sm.X[(s * D3 + k) * NR + c];
      sm.X[(3 * D3 + j) * NR + c] = v;
    }
    __syncthreads();
    // u = U^{-1} L_S^{-1} (b_u - ...)
    lds_forward_par<D3, true>(sm.S, sm.X + 3 * D3 * NR, NR, NR, 1, 0);
    lds_backward_par<D3, false>(sm.S, sm.X + 3 * D3 * NR, NR, NR, 1, 0);
    // q_s = L^{-T} (Z_s + G_s u)
    for (int idx = t; idx < 3 * D3 * NR; idx += nt) {
      const int s = idx / (D3 * NR), j = (idx / NR) % D3, c = idx % NR;
      double v = sm.X[idx];
      for (int k = 0; k < D3; ++k) v += sm.G[s][j * D3 + k] * sm.X[(3 * D3 + k) * NR + c];
      sm.X[idx] = v;
    }
    __syncthreads();
    lds_backward_par<D3, true>(sm.Mm, sm.X, NR, NR, 3, D3 * NR);
    // ---- C^K = A3 X_2 + tauDD - beta.n DD,  Cf^K = A3 X_f;  scatter or export
    for (int idx = t; idx < M * NR; idx += nt) {
      const int a = idx / NR, b = idx % NR;
      const int la = a / D2, ia = a % D2;
      const double* dpa = tb.DP + ((g.mu[la] * 4 + la) * D2 + ia) * D3;
      double v = 0;
      for (int j = 0; j < D3; ++j)
        v += dpa[j] * (g.n[la][0] * sm.X[j * NR + b] + g.n[la][1] * sm.X[(D3 + j) * NR + b] +
                       g.n[la][2] * sm.X[(2 * D3 + j) * NR + b] + g.T[la] * sm.X[(3 * D3 + j) * NR + b]);
      if (b == M) {
        if (Cfout)
          Cfout[(size_t)w * M + a] = v;
        else
          unsafeAtomicAdd(&F[(size_t)mesh.d_facebyele[4 * E + la] * D2 + ia], v);
        continue;
      }
      const int lb = b / D2, ib = b % D2;
      if (la == lb) v += (ia == ib ? g.T[la] : 0.0) - sm.bnDD[la][ia * D2 + ib];
      if (Cout) {
        Cout[((size_t)w * M + a) * M + b] = v;
        continue;
      }
      const size_t s1 = mesh.d_slot[16 * E + 4 * la + lb];
      if (la == lb)
        unsafeAtomicAdd(&H[(s1 * D2 + ia) * D2 + ib], v);
      else
        H[(s1 * D2 + ia) * D2 + ib] = v;
    }
    if (Xout)
      for (int idx = t; idx < N4 * NR; idx += nt) Xout[(size_t)w * N4 * NR + idx] = sm.X[idx];
  }
}

template <int D2>
__global__ void k_zero_diag_cd(const int* __restrict__ diag, int nfc, double* __restrict__ H, double* __restrict__ F) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)nfc * D2 * D2) return;
  const size_t f = i / (D2 * D2), e = i % (D2 * D2);
  H[(size_t)diag[f] * D2 * D2 + e] = 0.0;
  if (e < D2) F[f * D2 + e] = 0.0;
}

template <int K>
hdg_status run_cd(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c, const double* f,
                  const double* bvol, const double* bface, const double* tau, double* H, double* F, double* X,
                  const int* elems, int64_t n, double* Cout, double* Cfout, hipStream_t s) {
  using D = CdDims<K>;
  if (!Cout) {
    const size_t tot = (size_t)mesh->nfc * D::D2 * D::D2;
    k_zero_diag_cd<D::D2><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(mesh->d_diag, (int)mesh->nfc, H, F);
    HDG_CHECK_LAUNCH("k_zero_diag_cd");
  }
  if (n == 0) return HDG_OK;
  const int grid = (int)std::min<int64_t>(n, 8 * (int64_t)device_cu_count());
  timer_begin("k_condense_cd", s);
  k_condense_cd<K><<<grid, kCdThreads, 0, s>>>(*mesh, disc->dev, kappa, c, f, bvol, bface, tau, H, F, X, elems,
                                               (int)n, Cout, Cfout);
  timer_end("k_condense_cd", s);
  HDG_CHECK_LAUNCH("k_condense_cd");
  return HDG_OK;
}

hdg_status dispatch_cd(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                       const double* f, const double* bvol, const double* bface, const double* tau, double* H,
                       double* F, double* X, const int* elems, int64_t n, double* Cout, double* Cfout,
                       hipStream_t s, const char* who) {
  switch (disc->host.k) {
    case 0: return run_cd<0>(disc, mesh, kappa, c, f, bvol, bface, tau, H, F, X, elems, n, Cout, Cfout, s);
    case 1: return run_cd<1>(disc, mesh, kappa, c, f, bvol, bface, tau, H, F, X, elems, n, Cout, Cfout, s);
    case 2: return run_cd<2>(disc, mesh, kappa, c, f, bvol, bface, tau, H, F, X, elems, n, Cout, Cfout, s);
    case 3: return run_cd<3>(disc, mesh, kappa, c, f, bvol, bface, tau, H, F, X, elems, n, Cout, Cfout, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, std::string(who) + ": degrees 0..3 only");
}

// phi_l^K(qhat_r) = v_0 + B xhat_l(s_r, t_r), xhat_l the points of reference face l (eq 2.5)
__global__ void k_elem_face_points(hdg_mesh mesh, Tables tb, int nqd2, double* __restrict__ xyz) {
  const int64_t total = mesh.nelt * 4 * (int64_t)nqd2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t E = i / (4 * nqd2);
    const int l = (int)((i / nqd2) % 4), r = (int)(i % nqd2);
    const double s = tb.tri_pts[2 * r], tt = tb.tri_pts[2 * r + 1];
    double xi[3];
    switch (l) {
      case 0: xi[0] = s; xi[1] = tt; xi[2] = 0; break;
      case 1: xi[0] = s; xi[1] = 0; xi[2] = tt; break;
      case 2: xi[0] = 0; xi[1] = s; xi[2] = tt; break;
      default: xi[0] = s; xi[1] = tt; xi[2] = 1 - s - tt; break;
    }
    const int* el = mesh.d_elements + 4 * E;
    const double* p0 = mesh.d_coords + 3 * el[0];
    for (int d = 0; d < 3; ++d) {
      double x = p0[d];
      for (int m = 0; m < 3; ++m) x += (mesh.d_coords[3 * el[m + 1] + d] - p0[d]) * xi[m];
      xyz[3 * i + d] = x;
    }
  }
}

}  // namespace

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who);

}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_elem_face_qp_coords(const hdg_disc* disc, const hdg_mesh* mesh, double* d_xyz,
                                              void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_elem_face_qp_coords");
  if (st) return st;
  if (!d_xyz) return set_error(HDG_ERR_INVALID_ARG, "hdg_elem_face_qp_coords: NULL output");
  const int64_t total = mesh->nelt * 4 * (int64_t)disc->host.nqd2;
  k_elem_face_points<<<(unsigned)std::min<int64_t>((total + 255) / 256, 65535), 256, 0, (hipStream_t)stream>>>(
      *mesh, disc->dev, disc->host.nqd2, d_xyz);
  HDG_CHECK_LAUNCH("hdg_elem_face_qp_coords");
  return HDG_OK;
}

extern "C" hdg_status hdg_assemble_condense_cd(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                               const double* d_c, const double* d_f, const double* d_beta_vol,
                                               const double* d_beta_face, const double* d_tau, double* d_H,
                                               double* d_F, double* d_X, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_assemble_condense_cd");
  if (st) return st;
  if (!d_kappa || !d_c || !d_f || !d_beta_vol || !d_beta_face || !d_tau || !d_H || !d_F)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_assemble_condense_cd: NULL array");
  return dispatch_cd(disc, mesh, d_kappa, d_c, d_f, d_beta_vol, d_beta_face, d_tau, d_H, d_F, d_X, nullptr,
                     mesh->nelt, nullptr, nullptr, (hipStream_t)stream, "hdg_assemble_condense_cd");
}

extern "C" hdg_status hdg_export_local_cd(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                          const double* d_c, const double* d_f, const double* d_beta_vol,
                                          const double* d_beta_face, const double* d_tau, const int32_t* d_elems,
                                          int64_t n, double* d_C, double* d_Cf, double* d_X, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_export_local_cd");
  if (st) return st;
  if (!d_kappa || !d_c || !d_f || !d_beta_vol || !d_beta_face || !d_tau || !d_elems || !d_C || !d_Cf || n < 0)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_export_local_cd: NULL array or n < 0");
  return dispatch_cd(disc, mesh, d_kappa, d_c, d_f, d_beta_vol, d_beta_face, d_tau, nullptr, nullptr, d_X, d_elems,
                     n, d_C, d_Cf, (hipStream_t)stream, "hdg_export_local_cd");
}
