// Reconstruction of (q, u) from the face traces (eq 5.3, Section 6 "Reconstruction") and
// the local postprocess u* (eq 9.11), one wavefront per element.
//
// With the factors kept by the condensation (L L^T = M_{1/kappa}, Ls Ls^T = S, and f):
//   t_l = DP_l^T uhat_l,   r_s = sum_l n_{l s} t_l,          (r_s = (n_sDP)^T u_dK)
//   u   = S^{-1} ( f + sum_l T_l t_l + sum_s C_s M^{-1} r_s ),
//   q_s = M^{-1} ( C_s^T u - r_s ),
// which is the block elimination of A1 [q; u] = Af - A2 u_dK.
// Postprocess: S*_{ij} = int_K grad P_i . grad P_j = sum G_{hg} Shat^{hg} with
// G = det(B) B^{-1} B^{-T}; rhs_i = -sum_q |K| w_q kappa_q^{-1} (B^{-1} q_h(x_q)) . gradhat P_i;
// the hierarchical orthonormal basis makes the mean condition fix u*_1 = u_1, and the
// stiffness system is solved (Cholesky) on the remaining modes.
#include "tile.h"

namespace hdg {
namespace {

template <int K>
struct RecoverSmem {
  using Dm = Dims<K>;
  double L[Dm::D3 * Dm::D3];
  double LS[Dm::D3 * Dm::D3];
  double uh[4 * Dm::D2];
  double tl[4 * Dm::D3];
  double r[3 * Dm::D3];       // r_s, then M^{-1} r_s
  double x[3 * Dm::D3];       // right-hand sides of the q solves, then q
  double u[Dm::D3];
  double v[3 * Dm::D3];
  double y[3 * Dm::NQD];
  double Ss[Dm::D3P * Dm::D3P];
  double rs[Dm::D3P];
};

template <int N>
__device__ inline void solve_lower(const double* L, int ld, double* x, int stride) {
  for (int r = 0; r < N; ++r) {
    double s = x[r * stride];
    for (int k = 0; k < r; ++k) s -= L[r * ld + k] * x[k * stride];
    x[r * stride] = s / L[r * ld + r];
  }
}

template <int N>
__device__ inline void solve_upper_t(const double* L, int ld, double* x, int stride) {
  for (int r = N - 1; r >= 0; --r) {
    double s = x[r * stride];
    for (int k = r + 1; k < N; ++k) s -= L[k * ld + r] * x[k * stride];
    x[r * stride] = s / L[r * ld + r];
  }
}

// x <- A^{-1} x for an SPD block A, given either its lower Cholesky factor L (A = L L^T,
// two triangular solves) or, for the tile kernels' factor store, Ui = U^{-1} with
// A = U^T U stored as an upper matrix (two triangular products: A^{-1} = Ui Ui^T).
template <int N, bool INVERSE>
__device__ inline void spd_apply(const double* F, double* x) {
  if constexpr (INVERSE) {
    double y[N];
    for (int i = 0; i < N; ++i) {  // y = Ui^T x
      double s = 0;
      for (int j = 0; j <= i; ++j) s += F[j * N + i] * x[j];
      y[i] = s;
    }
    for (int i = 0; i < N; ++i) {  // x = Ui y
      double s = 0;
      for (int j = i; j < N; ++j) s += F[i * N + j] * y[j];
      x[i] = s;
    }
  } else {
    solve_lower<N>(F, N, x, 1);
    solve_upper_t<N>(F, N, x, 1);
  }
}

template <int K, bool TILE>
__global__ void __launch_bounds__(64) k_recover(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                const double* __restrict__ tau, const double* __restrict__ factors,
                                                const double* __restrict__ uhat, double* __restrict__ qout,
                                                double* __restrict__ uout, double* __restrict__ usout) {
  using Dm = Dims<K>;
  constexpr int D3 = Dm::D3, D2 = Dm::D2, NQD = Dm::NQD, D3P = Dm::D3P;
  __shared__ RecoverSmem<K> sm;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int E = blockIdx.x; E < mesh.nelt; E += gridDim.x) {
    ElemGeom g;
    load_geometry(E, mesh, tau, g);
    constexpr int TT = (D3 + 3) / 4, NU = TT * (TT + 1) / 2;
    constexpr int FLEN = TILE ? (2 * NU + TT) * 16 : D3 * (D3 + 1) + D3;
    const double* fa = factors + (size_t)E * FLEN;
    for (int idx = t; idx < D3 * D3; idx += nt) {
      const int i = idx / D3, j = idx % D3;
      if constexpr (TILE) {
        // upper inverses U^{-1}, Us^{-1} stored as packed upper 4x4 tiles: entry (i, j), j >= i
        if (j < i) continue;
        const int o = utile(i / 4, j / 4, TT) * 16 + (i % 4) * 4 + (j % 4);
        sm.L[idx] = fa[o];
        sm.LS[idx] = fa[NU * 16 + o];
      } else {
        if (j > i) continue;
        sm.L[idx] = fa[i * (i + 1) / 2 + j];
        sm.LS[idx] = fa[D3 * (D3 + 1) / 2 + i * (i + 1) / 2 + j];
      }
    }
    for (int idx = t; idx < 4 * D2; idx += nt)
      sm.uh[idx] = uhat[(size_t)mesh.d_facebyele[4 * E + idx / D2] * D2 + idx % D2];
    __syncthreads();
    // t_l = DP_l^T uhat_l
    for (int idx = t; idx < 4 * D3; idx += nt) {
      const int l = idx / D3, j = idx % D3;
      const double* dp = tb.DP + (size_t)((g.mu[l] * 4 + l) * D2) * D3;
      double s = 0;
      for (int i = 0; i < D2; ++i) s += dp[i * D3 + j] * sm.uh[l * D2 + i];
      sm.tl[idx] = s;
    }
    __syncthreads();
    // r_s and the right-hand side pieces
    for (int idx = t; idx < 3 * D3; idx += nt) {
      const int s = idx / D3, j = idx % D3;
      double v = 0;
      for (int l = 0; l < 4; ++l) v += g.n[l][s] * sm.tl[l * D3 + j];
      sm.r[idx] = v;
      sm.x[idx] = v;
    }
    __syncthreads();
    // x_s <- M^{-1} r_s  (three columns)
    if (t < 3) {
      spd_apply<D3, TILE>(sm.L, sm.x + t * D3);
    }
    __syncthreads();
    // v_h = sum_s a[s][h] (M^{-1} r_s)
    for (int idx = t; idx < 3 * D3; idx += nt) {
      const int h = idx / D3, j = idx % D3;
      sm.v[idx] = g.a[0][h] * sm.x[j] + g.a[1][h] * sm.x[D3 + j] + g.a[2][h] * sm.x[2 * D3 + j];
    }
    __syncthreads();
    // rhs_u = f + sum_l T_l t_l + sum_h Chat^h v_h
    for (int i = t; i < D3; i += nt) {
      double s = TILE ? fa[(2 * NU + i / 4) * 16 + (i % 4) * 4] : fa[D3 * (D3 + 1) + i];
      for (int l = 0; l < 4; ++l) s += g.T[l] * sm.tl[l * D3 + i];
      for (int h = 0; h < 3; ++h)
        for (int j = 0; j < D3; ++j) s += tb.Chat[(h * D3 + i) * D3 + j] * sm.v[h * D3 + j];
      sm.u[i] = s;
    }
    __syncthreads();
    if (t == 0) {
      spd_apply<D3, TILE>(sm.LS, sm.u);
    }
    __syncthreads();
    // x_s = C_s^T u - r_s with (C_s^T u)_i = sum_h a[s][h] sum_j Chat^h[j][i] u_j
    for (int idx = t; idx < 3 * D3; idx += nt) {
      const int h = idx / D3, i = idx % D3;
      double s = 0;
      for (int j = 0; j < D3; ++j) s += tb.Chat[(h * D3 + j) * D3 + i] * sm.u[j];
      sm.v[idx] = s;
    }
    __syncthreads();
    for (int idx = t; idx < 3 * D3; idx += nt) {
      const int s = idx / D3, i = idx % D3;
      sm.x[idx] = g.a[s][0] * sm.v[i] + g.a[s][1] * sm.v[D3 + i] + g.a[s][2] * sm.v[2 * D3 + i] - sm.r[idx];
    }
    __syncthreads();
    if (t < 3) {
      spd_apply<D3, TILE>(sm.L, sm.x + t * D3);
    }
    __syncthreads();
    for (int idx = t; idx < 3 * D3; idx += nt) qout[(size_t)E * 3 * D3 + idx] = sm.x[idx];
    for (int i = t; i < D3; i += nt) uout[(size_t)E * D3 + i] = sm.u[i];
    if (usout) {
      // y_h(q) = |K| w_q kappa_q^{-1} (B^{-1} q_h(x_q))_h, with B^{-1} = a^T / det
      for (int q = t; q < NQD; q += nt) {
        double qh[3] = {0, 0, 0};
        for (int j = 0; j < D3; ++j) {
          const double p = tb.P[q * D3 + j];
          qh[0] += sm.x[j] * p;
          qh[1] += sm.x[D3 + j] * p;
          qh[2] += sm.x[2 * D3 + j] * p;
        }
        const double wq = g.vol * tb.vol_w[q] / kappa[(size_t)E * NQD + q] / g.det;
        for (int h = 0; h < 3; ++h)
          sm.y[h * NQD + q] = wq * (g.a[0][h] * qh[0] + g.a[1][h] * qh[1] + g.a[2][h] * qh[2]);
      }
      // G = a^T a / det
      double G[3][3];
      for (int h = 0; h < 3; ++h)
        for (int k = 0; k < 3; ++k)
          G[h][k] = (g.a[0][h] * g.a[0][k] + g.a[1][h] * g.a[1][k] + g.a[2][h] * g.a[2][k]) / g.det;
      const double cf[6] = {G[0][0], G[1][1], G[2][2], G[0][1], G[0][2], G[1][2]};
      for (int idx = t; idx < D3P * D3P; idx += nt) {
        double s = 0;
        for (int p = 0; p < 6; ++p) s += cf[p] * tb.Shat[p * D3P * D3P + idx];
        sm.Ss[idx] = s;
      }
      __syncthreads();
      for (int i = t; i < D3P; i += nt) {
        double s = 0;
        for (int h = 0; h < 3; ++h)
          for (int q = 0; q < NQD; ++q) s -= sm.y[h * NQD + q] * tb.P1g[(h * NQD + q) * D3P + i];
        sm.rs[i] = s;
      }
      __syncthreads();
      // Cholesky of S* restricted to modes 2..d3p, then the solve
      lds_cholesky<D3P - 1>(sm.Ss + D3P + 1, D3P);
      if (t == 0) {
        solve_lower<D3P - 1>(sm.Ss + D3P + 1, D3P, sm.rs + 1, 1);
        solve_upper_t<D3P - 1>(sm.Ss + D3P + 1, D3P, sm.rs + 1, 1);
        sm.rs[0] = sm.u[0];
      }
      __syncthreads();
      for (int i = t; i < D3P; i += nt) usout[(size_t)E * D3P + i] = sm.rs[i];
    }
    __syncthreads();
  }
}

template <int K>
hdg_status run_recover(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* tau,
                       const double* factors, const double* uhat, double* q, double* u, double* us, hipStream_t s) {
  const int grid = (int)std::min<int64_t>(mesh->nelt, 1 << 20);
  k_recover<K, (K >= 1 && K <= 3)><<<grid, 64, 0, s>>>(*mesh, disc->dev, kappa, tau, factors, uhat, q, u, us);
  HDG_CHECK_LAUNCH("k_recover");
  return HDG_OK;
}

}  // namespace

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who);

}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_recover(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                  const double* d_tau, const double* d_factors, const double* d_uhat, double* d_q,
                                  double* d_u, double* d_ustar, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_recover");
  if (st) return st;
  if (!d_kappa || !d_tau || !d_factors || !d_uhat || !d_q || !d_u)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_recover: NULL array");
  hipStream_t s = (hipStream_t)stream;
  switch (disc->host.k) {
    case 0: return run_recover<0>(disc, mesh, d_kappa, d_tau, d_factors, d_uhat, d_q, d_u, d_ustar, s);
    case 1: return run_recover<1>(disc, mesh, d_kappa, d_tau, d_factors, d_uhat, d_q, d_u, d_ustar, s);
    case 2: return run_recover<2>(disc, mesh, d_kappa, d_tau, d_factors, d_uhat, d_q, d_u, d_ustar, s);
    case 3: return run_recover<3>(disc, mesh, d_kappa, d_tau, d_factors, d_uhat, d_q, d_u, d_ustar, s);
    case 4: return run_recover<4>(disc, mesh, d_kappa, d_tau, d_factors, d_uhat, d_q, d_u, d_ustar, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_recover: unsupported degree");
}
