// Local projections and the superconvergence diagnostics (Section 9, "Local L2 projections"
// and "HDG projection"; eq 9.12, 9.13, 10.2).
//
// Trace projection (eq 9.12).  With the orthonormal face basis the face mass matrix in the
// normalised weights is the identity, so P v on face e has the coefficients
//     (P v)_i = sum_r w_r D_i(qhat_r) v(y_r),   y_r = phi_e(qhat_r)
// (the formula of eq 6.3 with ((w.D)^T D)^{-1} = I).  k_face_moments computes these moments
// for several fields at once, one thread per (face, field, mode).
//
// HDG projection (eq 9.13).  The unit mass matrix of K in the orthonormal hierarchical basis
// is |K| I, so the volume equations fix the modes below the top degree directly:
//     (Pi q_s)_i = sum_q w_q q_s(x_q) P_i(x_q),  (Pi u)_i likewise,  i < d3 - d2.
// The face equations of face l (d2 each), in the normalised face weights, read
//     sum_s n_ls DP_l (Pi q_s) + T_l DP_l (Pi u) = sum_c w_lc rho_{e,c},
// with w_l = (n_lx, n_ly, n_lz, T_l), T_l = tau_l |e_l|, DP_l = DP_{mu(K,l),l} (eq 4.10) and
// rho_e the face moments of (q_x, q_y, q_z, u).  Splitting DP_l = [DP_l^lo | A_l] (the last d2
// columns) and X = the top modes of the four fields (4 x d2):
//     A_l (sum_c w_lc X_c) = sum_c w_lc (rho_{e,c} - DP_l^lo (Pi v_c)^lo) =: r_l,
// so sum_c w_lc X_c = A_l^{-1} r_l =: y_l for l = 1..4, i.e. W X = Y with the 4 x 4 matrix W
// of rows w_l.  A_l^{-1} is a reference table (24 of them); W is invertible exactly when tau
// does not vanish on all four faces (its determinant is +-(sum_l T_l) det[n_1 n_2 n_3], since
// sum_l n_l = 0).  So the 4 d3 x 4 d3 system of the paper becomes four d2 x d2 table products
// and one 4 x 4 solve per element.
//
// Norms of eq 10.2 (squared): ||Pi u - u_h||_K^2 = |K| sum_i (Pi u - u_h)_i^2 and
// ||P u - uhat||_e^2 = |e| sum_i (..)_i^2 (orthonormal bases), ||u||_K^2 and ||u||_e^2 by the
// quadrature rules of the discretisation; fixed-order two-stage reductions.
#include <algorithm>

#include "device_common.h"

namespace hdg {
namespace {

// rho[f][c][i] = sum_r tri_w[r] D[r][i] v[f][r][c] for the n faces of the caller's list.
__global__ void k_face_moments(const double* __restrict__ vals, int ncomp, int nqd2, int d2, int64_t n,
                               const double* __restrict__ tri_w, const double* __restrict__ D,
                               double* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int per = ncomp * d2;
  if (t >= n * per) return;
  const int64_t f = t / per;
  const int rem = (int)(t - f * per), c = rem / d2, i = rem % d2;
  const double* v = vals + f * (int64_t)nqd2 * ncomp + c;
  double s = 0.0;
  for (int r = 0; r < nqd2; ++r) s = fma(tri_w[r] * D[r * d2 + i], v[(int64_t)r * ncomp], s);
  out[t] = s;
}

// The common four-field case (q_x, q_y, q_z, u): one thread per (face, mode), the four fields
// of a point read as one 32-byte load.
__global__ void k_face_moments4(const double* __restrict__ vals, int nqd2, int d2, int64_t n,
                                const double* __restrict__ tri_w, const double* __restrict__ D,
                                double* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * d2) return;
  const int64_t f = t / d2;
  const int i = (int)(t - f * d2);
  const double4* v = reinterpret_cast<const double4*>(vals) + f * nqd2;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll 4
  for (int r = 0; r < nqd2; ++r) {
    const double w = tri_w[r] * D[r * d2 + i];
    const double4 x = v[r];
    a0 = fma(w, x.x, a0);
    a1 = fma(w, x.y, a1);
    a2 = fma(w, x.z, a2);
    a3 = fma(w, x.w, a3);
  }
  double* o = out + f * 4 * d2 + i;
  o[0] = a0;
  o[d2] = a1;
  o[2 * d2] = a2;
  o[3 * d2] = a3;
}

// A tile of ET elements per 256-thread workgroup (persistent over tiles).  The table
// w_q P_i(x_q) of the low modes is staged in LDS once per workgroup; every phase spreads its
// (element, index) tasks over all threads:
//   low modes   thread (e, i): one pass over the points with the four fields of a point read
//               as one 32-byte load, four accumulators;
//   face rows   thread (e, l, i): r_l,i = sum_c w_lc (rho_{e_l,c,i} - DP_l^lo,i . v_c^lo);
//   W^{-1}      thread e: Gauss-Jordan of the 4 x 4 matrix W;
//   y, top      thread (e, l, i): y_l = A_l^{-1} r_l, then thread (e, c, i): X_c = (W^{-1} Y)_c;
//   output      thread (e, c, i) over the whole [3 + 1][d3] block of the tile (coalesced).
constexpr int kProjThreads = 256;

template <int K>
struct ProjTile {
  static constexpr int D3 = dim3(K), D2 = dim2(K), NQD = (K + 2) * (K + 2) * (K + 2), LOW = D3 - D2;
  static constexpr int ET = LOW > 0 ? (kProjThreads / LOW > 32 ? 32 : kProjThreads / LOW) : 32;
  static constexpr int L1 = LOW > 0 ? LOW : 1;
  static constexpr size_t lds_bytes() {
    return 8 * ((size_t)NQD * L1 + ET * 4 * L1 + ET * 4 * D2 + ET * 16) + 8 * 4 * ET;
  }
};

template <int K>
__global__ void __launch_bounds__(kProjThreads) k_hdg_projection(hdg_mesh mesh, Tables tb, const double* __restrict__ tau,
                                                                 const double* __restrict__ qu_vol,
                                                                 const double* __restrict__ rho,
                                                                 double* __restrict__ Pq, double* __restrict__ Pu) {
  using PT = ProjTile<K>;
  constexpr int D3 = PT::D3, D2 = PT::D2, NQD = PT::NQD, LOW = PT::LOW, ET = PT::ET, L1 = LOW > 0 ? LOW : 1;
  __shared__ double s_wp[NQD * L1];      // w_q P_i(x_q), i < LOW
  __shared__ double s_lo[ET][4][L1];     // low modes of (q_x, q_y, q_z, u)
  __shared__ double s_r[ET][4][D2];      // r_l, then y_l
  __shared__ double s_w[ET][4][4];       // W, then W^{-1}
  __shared__ int s_f[ET][4], s_mu[ET][4];
  const int tid = threadIdx.x;
  for (int j = tid; j < NQD * LOW; j += kProjThreads) {
    const int q = j / LOW, i = j % LOW;
    s_wp[j] = tb.vol_w[q] * tb.P[q * D3 + i];
  }
  const int64_t ntile = (mesh.nelt + ET - 1) / ET;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t E0 = tile * ET;
    const int ne = (int)min<int64_t>(ET, mesh.nelt - E0);
    __syncthreads();
    for (int t = tid; t < 4 * ne; t += kProjThreads) {
      const int e = t >> 2, l = t & 3;
      const size_t E = (size_t)(E0 + e);
      const double* n = mesh.d_normals + 12 * E + 3 * l;
      const double n0 = n[0], n1 = n[1], n2 = n[2];
      s_w[e][l][0] = n0;
      s_w[e][l][1] = n1;
      s_w[e][l][2] = n2;
      s_w[e][l][3] = tau[4 * E + l] * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
      s_f[e][l] = mesh.d_facebyele[4 * E + l];
      s_mu[e][l] = mesh.d_perm[4 * E + l] - 1;
    }
    // modes below the top degree: the L2 moments (unit mass |K| I)
    for (int t = tid; t < LOW * ne; t += kProjThreads) {
      const int e = t / LOW, i = t % LOW;
      const double4* v = reinterpret_cast<const double4*>(qu_vol + (size_t)(E0 + e) * NQD * 4);
      double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll 8
      for (int q = 0; q < NQD; ++q) {
        const double w = s_wp[q * L1 + i];
        const double4 x = v[q];
        a0 = fma(w, x.x, a0);
        a1 = fma(w, x.y, a1);
        a2 = fma(w, x.z, a2);
        a3 = fma(w, x.w, a3);
      }
      s_lo[e][0][i] = a0;
      s_lo[e][1][i] = a1;
      s_lo[e][2][i] = a2;
      s_lo[e][3][i] = a3;
    }
    __syncthreads();
    // r_l = sum_c w_lc (rho_{e,c} - DP_l^lo v_c^lo)
    for (int t = tid; t < 4 * D2 * ne; t += kProjThreads) {
      const int e = t / (4 * D2), li = t % (4 * D2), l = li / D2, i = li % D2;
      const double* dp = tb.DP + ((size_t)(s_mu[e][l] * 4 + l) * D2 + i) * D3;
      const double* rh = rho + (size_t)s_f[e][l] * 4 * D2 + i;
      double r = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double sc = rh[c * D2];
        for (int j = 0; j < LOW; ++j) sc = fma(-dp[j], s_lo[e][c][j], sc);
        r = fma(s_w[e][l][c], sc, r);
      }
      s_r[e][l][i] = r;
    }
    __syncthreads();
    // W^{-1} (one thread per element; Gauss-Jordan with partial pivoting)
    for (int e = tid; e < ne; e += kProjThreads) {
      double a[4][8];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          a[i][j] = s_w[e][i][j];
          a[i][4 + j] = i == j ? 1.0 : 0.0;
        }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        int piv = c;
#pragma unroll
        for (int r = c + 1; r < 4; ++r)
          if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (r == piv && r != c) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const double x = a[c][j];
              a[c][j] = a[r][j];
              a[r][j] = x;
            }
          }
        const double inv = 1.0 / a[c][c];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[c][j] *= inv;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (r != c) {
            const double f = a[r][c];
#pragma unroll
            for (int j = 0; j < 8; ++j) a[r][j] = fma(-f, a[c][j], a[r][j]);
          }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) s_w[e][i][j] = a[i][4 + j];
    }
    // y_l = A_l^{-1} r_l (kept in registers until every r has been read)
    double yv[(4 * D2 * ET + kProjThreads - 1) / kProjThreads];
    {
      int u = 0;
      for (int t = tid; t < 4 * D2 * ne; t += kProjThreads, ++u) {
        const int e = t / (4 * D2), li = t % (4 * D2), l = li / D2, i = li % D2;
        const double* ai = tb.DPtopinv + ((size_t)(s_mu[e][l] * 4 + l) * D2 + i) * D2;
        double y = 0.0;
        for (int j = 0; j < D2; ++j) y = fma(ai[j], s_r[e][l][j], y);
        yv[u] = y;
      }
    }
    __syncthreads();
    {
      int u = 0;
      for (int t = tid; t < 4 * D2 * ne; t += kProjThreads, ++u) {
        const int e = t / (4 * D2), li = t % (4 * D2);
        s_r[e][li / D2][li % D2] = yv[u];
      }
    }
    __syncthreads();
    // outputs: per element [3][D3] of Pq and [D3] of Pu, low modes then top modes
    for (int t = tid; t < 4 * D3 * ne; t += kProjThreads) {
      const int e = t / (4 * D3), ci = t % (4 * D3), c = ci / D3, i = ci % D3;
      double v;
      if (i < LOW) {
        v = s_lo[e][c][i];
      } else {
        v = 0.0;
#pragma unroll
        for (int l = 0; l < 4; ++l) v = fma(s_w[e][c][l], s_r[e][l][i - LOW], v);
      }
      const size_t E = (size_t)(E0 + e);
      if (c < 3)
        Pq[(E * 3 + c) * D3 + i] = v;
      else
        Pu[E * D3 + i] = v;
    }
  }
}

// Squared norms of eq 10.2, one partial per block (fixed grid), then one block sums them.
// out[0] = sum_K |K| |Pu - uh|^2, out[1] = sum_K |K| sum_q w_q u(x_q)^2,
// out[2] = sum_e |e|^2 |Puhat - uhat|^2, out[3] = sum_e |e|^2 sum_r w_r u(y_r)^2.
constexpr int kNormThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kNormThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kNormThreads)
k_norm_partials(const double* __restrict__ vol, const double* __restrict__ area, int64_t nelt, int64_t nfc, int d3,
                int d2, int nqd, int nqd2, const double* __restrict__ vol_w, const double* __restrict__ tri_w,
                const double* __restrict__ Pu, const double* __restrict__ uh, const double* __restrict__ u_vol,
                const double* __restrict__ Pt, const double* __restrict__ uhat, const double* __restrict__ u_face,
                double* __restrict__ part) {
  __shared__ double sh[kNormThreads];
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  const int64_t stride = (int64_t)gridDim.x * kNormThreads;
  for (int64_t K = blockIdx.x * (int64_t)kNormThreads + threadIdx.x; K < nelt; K += stride) {
    double a = 0, b = 0;
    for (int i = 0; i < d3; ++i) {
      const double d = Pu[K * d3 + i] - uh[K * d3 + i];
      a = fma(d, d, a);
    }
    if (u_vol)
      for (int q = 0; q < nqd; ++q) {
        const double v = u_vol[K * nqd + q];
        b = fma(vol_w[q] * v, v, b);
      }
    s0 = fma(vol[K], a, s0);
    s1 = fma(vol[K], b, s1);
  }
  for (int64_t f = blockIdx.x * (int64_t)kNormThreads + threadIdx.x; f < nfc; f += stride) {
    double a = 0, b = 0;
    for (int i = 0; i < d2; ++i) {
      const double d = Pt[f * d2 + i] - uhat[f * d2 + i];
      a = fma(d, d, a);
    }
    if (u_face)
      for (int r = 0; r < nqd2; ++r) {
        const double v = u_face[f * nqd2 + r];
        b = fma(tri_w[r] * v, v, b);
      }
    const double e2 = area[f] * area[f];
    s2 = fma(e2, a, s2);
    s3 = fma(e2, b, s3);
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  s3 = block_sum(s3, sh);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x + 0] = s0;
    part[4 * blockIdx.x + 1] = s1;
    part[4 * blockIdx.x + 2] = s2;
    part[4 * blockIdx.x + 3] = s3;
  }
}

__global__ void __launch_bounds__(kNormThreads) k_norm_final(const double* __restrict__ part, int nb,
                                                             double* __restrict__ out) {
  __shared__ double sh[kNormThreads];
  for (int j = 0; j < 4; ++j) {
    double s = 0;
    for (int b = threadIdx.x; b < nb; b += kNormThreads) s += part[4 * b + j];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[j] = s;
  }
}

int norm_blocks(int64_t nelt, int64_t nfc) {
  const int64_t n = std::max(nelt, nfc);
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kNormThreads - 1) / kNormThreads, 1024));
}

template <int K>
void launch_hdg_projection(const hdg_disc* disc, const hdg_mesh* mesh, const double* tau, const double* qu_vol,
                           const double* rho, double* Pq, double* Pu, hipStream_t s) {
  using PT = ProjTile<K>;
  const int64_t ntile = (mesh->nelt + PT::ET - 1) / PT::ET;
  // as many resident workgroups per compute unit as 160 KB of LDS allows (at most 8)
  const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / PT::lds_bytes()));
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ntile, (int64_t)per_cu * device_cu_count()));
  timer_begin("k_hdg_projection", s);
  k_hdg_projection<K><<<grid, kProjThreads, 0, s>>>(*mesh, disc->dev, tau, qu_vol, rho, Pq, Pu);
  timer_end("k_hdg_projection", s);
}

}  // namespace

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who);

}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_project_trace(const hdg_disc* disc, const hdg_mesh* mesh, int64_t n, int ncomp,
                                        const double* d_vals, double* d_out, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_project_trace");
  if (st) return st;
  if (!d_vals || !d_out || n < 0 || ncomp < 1 || ncomp > 8)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_project_trace: NULL array, n < 0 or ncomp outside 1..8");
  if (n == 0) return HDG_OK;
  const auto& h = disc->host;
  const int64_t tot = n * ncomp * h.d2;
  hipStream_t s = (hipStream_t)stream;
  timer_begin("k_face_moments", s);
  if (ncomp == 4 && ((uintptr_t)d_vals & 31) == 0) {
    const int64_t nt = n * h.d2;
    k_face_moments4<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(d_vals, h.nqd2, h.d2, n, disc->dev.tri_w,
                                                                   disc->dev.D, d_out);
  } else {
    k_face_moments<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(d_vals, ncomp, h.nqd2, h.d2, n, disc->dev.tri_w,
                                                                   disc->dev.D, d_out);
  }
  timer_end("k_face_moments", s);
  HDG_CHECK_LAUNCH("k_face_moments");
  return HDG_OK;
}

extern "C" hdg_status hdg_project_hdg_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, size_t* bytes) {
  if (!disc || !mesh || !bytes) return set_error(HDG_ERR_INVALID_ARG, "hdg_project_hdg_workspace_size: NULL argument");
  *bytes = (size_t)mesh->nfc * 4 * disc->host.d2 * sizeof(double);
  return HDG_OK;
}

extern "C" hdg_status hdg_project_hdg(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_tau,
                                      const double* d_qu_vol, const double* d_qu_face, double* d_Pq, double* d_Pu,
                                      void* d_ws, size_t ws_bytes, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_project_hdg");
  if (st) return st;
  if (!d_tau || !d_qu_vol || !d_qu_face || !d_Pq || !d_Pu)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_project_hdg: NULL array");
  if (((uintptr_t)d_qu_vol & 31) != 0)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_project_hdg: d_qu_vol must be 32-byte aligned");
  size_t need = 0;
  hdg_project_hdg_workspace_size(disc, mesh, &need);
  if (!d_ws || ws_bytes < need) return set_error(HDG_ERR_WORKSPACE, "hdg_project_hdg: workspace too small");
  double* rho = (double*)d_ws;
  st = hdg_project_trace(disc, mesh, mesh->nfc, 4, d_qu_face, rho, stream);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  switch (disc->host.k) {
    case 0: launch_hdg_projection<0>(disc, mesh, d_tau, d_qu_vol, rho, d_Pq, d_Pu, s); break;
    case 1: launch_hdg_projection<1>(disc, mesh, d_tau, d_qu_vol, rho, d_Pq, d_Pu, s); break;
    case 2: launch_hdg_projection<2>(disc, mesh, d_tau, d_qu_vol, rho, d_Pq, d_Pu, s); break;
    case 3: launch_hdg_projection<3>(disc, mesh, d_tau, d_qu_vol, rho, d_Pq, d_Pu, s); break;
    case 4: launch_hdg_projection<4>(disc, mesh, d_tau, d_qu_vol, rho, d_Pq, d_Pu, s); break;
    default: return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_project_hdg: unsupported degree");
  }
  HDG_CHECK_LAUNCH("k_hdg_projection");
  return HDG_OK;
}

extern "C" hdg_status hdg_superconvergence_norms_workspace_size(const hdg_mesh* mesh, size_t* bytes) {
  if (!mesh || !bytes) return set_error(HDG_ERR_INVALID_ARG, "hdg_superconvergence_norms_workspace_size: NULL");
  *bytes = (size_t)norm_blocks(mesh->nelt, mesh->nfc) * 4 * sizeof(double);
  return HDG_OK;
}

extern "C" hdg_status hdg_superconvergence_norms(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_Pu,
                                                 const double* d_uh, const double* d_u_vol, const double* d_Puhat,
                                                 const double* d_uhat, const double* d_u_face, double* d_out,
                                                 void* d_ws, size_t ws_bytes, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_superconvergence_norms");
  if (st) return st;
  if (!d_Pu || !d_uh || !d_Puhat || !d_uhat || !d_out || !mesh->d_volume || !mesh->d_area)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_superconvergence_norms: NULL array");
  size_t need = 0;
  hdg_superconvergence_norms_workspace_size(mesh, &need);
  if (!d_ws || ws_bytes < need)
    return set_error(HDG_ERR_WORKSPACE, "hdg_superconvergence_norms: workspace too small");
  const auto& h = disc->host;
  const int nb = norm_blocks(mesh->nelt, mesh->nfc);
  hipStream_t s = (hipStream_t)stream;
  k_norm_partials<<<nb, kNormThreads, 0, s>>>(mesh->d_volume, mesh->d_area, mesh->nelt, mesh->nfc, h.d3, h.d2, h.nqd,
                                              h.nqd2, disc->dev.vol_w, disc->dev.tri_w, d_Pu, d_uh, d_u_vol, d_Puhat,
                                              d_uhat, d_u_face, (double*)d_ws);
  k_norm_final<<<1, kNormThreads, 0, s>>>((const double*)d_ws, nb, d_out);
  HDG_CHECK_LAUNCH("k_norm_partials / k_norm_final");
  return HDG_OK;
}
