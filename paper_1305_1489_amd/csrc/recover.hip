// Reconstruction of (q, u) from the face traces (eq 5.3, Section 6 "Reconstruction"),
// one wavefront per element (four at degrees 5 and 6), every step spread over its lanes.
// The local postprocess u* (eq 9.11) runs afterwards in its own kernel (postprocess.hip).
//
// With the factors kept by the condensation (M = M_{1/kappa}, S the u-Schur complement,
// and f):
//   t_l = DP_l^T uhat_l,   r_s = sum_l n_{l s} t_l,          (r_s = (n_sDP)^T u_dK)
//   u   = S^{-1} ( f + sum_l T_l t_l + sum_s C_s M^{-1} r_s ),
//   q_s = M^{-1} ( C_s^T u - r_s ),
// which is the block elimination of A1 [q; u] = Af - A2 u_dK.  The tile kernels (k = 1..3)
// store the inverse upper Cholesky factors U^{-1}, Us^{-1} (A^{-1} = U^{-1} U^{-T}, two
// triangular products); the per-element kernel (k = 0, 4) stores the lower factors.
// Postprocess: S*_{ij} = int_K grad P_i . grad P_j = sum G_{hg} Shat^{hg} with
// G = det(B) B^{-1} B^{-T}; rhs_i = -sum_q |K| w_q kappa_q^{-1} (B^{-1} q_h(x_q)) . gradhat P_i;
// the hierarchical orthonormal basis makes the mean condition fix u*_1 = u_1, and the
// stiffness system is solved (Cholesky) on the remaining modes.
#include "tile.h"

namespace hdg {

hdg_status launch_postprocess(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* tau,
                              const double* q, const double* u, const double* factors, double* us, hipStream_t s);

namespace {

template <int K>
struct RecoverSmem {
  using Dm = Dims<K>;
  double L[Dm::D3 * Dm::D3];
  double LS[Dm::D3 * Dm::D3];
  double uh[4 * Dm::D2];
  double tl[4 * Dm::D3];
  double r[3 * Dm::D3];    // r_s
  double x[3 * Dm::D3];    // right-hand sides of the M solves, then their solutions
  double tmp[3 * Dm::D3];
  double u[Dm::D3];
  double v[3 * Dm::D3];
};

// ---- wavefront-parallel dense kernels on LDS data (all lanes of the block take part)

// X <- L^{-1} X then X <- L^{-T} X for ncols columns of length N (column stride N).
template <int N>
__device__ inline void par_chol_solve(const double* L, int ld, double* X, int ncols) {
  const int t = threadIdx.x, nt = blockDim.x;
  for (int j = 0; j < N; ++j) {
    for (int c = t; c < ncols; c += nt) X[c * N + j] /= L[j * ld + j];
    __syncthreads();
    const int w = N - j - 1;
    for (int p = t; p < w * ncols; p += nt) {
      const int c = p / w, i = j + 1 + p % w;
      X[c * N + i] -= L[i * ld + j] * X[c * N + j];
    }
    __syncthreads();
  }
  for (int j = N - 1; j >= 0; --j) {
    for (int c = t; c < ncols; c += nt) X[c * N + j] /= L[j * ld + j];
    __syncthreads();
    for (int p = t; p < j * ncols; p += nt) {
      const int c = p / j, i = p % j;
      X[c * N + i] -= L[j * ld + i] * X[c * N + j];
    }
    __syncthreads();
  }
}

// X <- Ui (Ui^T X) for ncols columns; Ui upper (row-major N x N), tmp as large as X.
template <int N>
__device__ inline void par_inverse_apply(const double* Ui, double* X, double* tmp, int ncols) {
  const int t = threadIdx.x, nt = blockDim.x;
  for (int p = t; p < N * ncols; p += nt) {
    const int c = p / N, i = p % N;
    double s = 0;
    for (int j = 0; j <= i; ++j) s += Ui[j * N + i] * X[c * N + j];
    tmp[p] = s;
  }
  __syncthreads();
  for (int p = t; p < N * ncols; p += nt) {
    const int c = p / N, i = p % N;
    double s = 0;
    for (int j = i; j < N; ++j) s += Ui[i * N + j] * tmp[c * N + j];
    X[p] = s;
  }
  __syncthreads();
}

template <int N, bool TILE>
__device__ inline void spd_apply(const double* F, double* X, double* tmp, int ncols) {
  if constexpr (TILE)
    par_inverse_apply<N>(F, X, tmp, ncols);
  else
    par_chol_solve<N>(F, N, X, ncols);
}

// Threads per element of the per-element reconstruction: one wavefront, four at degrees 5
// and 6, whose two d3 x d3 factors in LDS (125 KB at k = 6) leave room for one element per CU.
constexpr int recover_threads(int k) { return k >= 5 ? 256 : 64; }

template <int K, bool TILE>
__global__ void __launch_bounds__(recover_threads(K)) k_recover(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                const double* __restrict__ tau, const double* __restrict__ factors,
                                                const double* __restrict__ uhat, double* __restrict__ qout,
                                                double* __restrict__ uout) {
  using Dm = Dims<K>;
  constexpr int D3 = Dm::D3, D2 = Dm::D2, NQD = Dm::NQD, D3P = Dm::D3P;
  constexpr int TT = (D3 + 3) / 4, NU = TT * (TT + 1) / 2;
  constexpr int FLEN = TILE ? (2 * NU + TT) * 16 + kGeoRecord : D3 * (D3 + 1) + D3;
  __shared__ RecoverSmem<K> sm;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int E = blockIdx.x; E < mesh.nelt; E += gridDim.x) {
    // element geometry in LDS (indexed at run time below; registers would spill)
    __shared__ ElemGeom sg;
    if (t == 0) load_geometry(E, mesh, tau, sg);
    __syncthreads();
    const ElemGeom& g = sg;
    const double* fa = factors + (size_t)E * FLEN;
    for (int idx = t; idx < D3 * D3; idx += nt) {
      const int i = idx / D3, j = idx % D3;
      if constexpr (TILE) {
        // U^{-1}, Us^{-1}: packed upper 4x4 tiles, entry (i, j) with j >= i
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
    // r_s
    for (int idx = t; idx < 3 * D3; idx += nt) {
      const int s = idx / D3, j = idx % D3;
      double v = 0;
      for (int l = 0; l < 4; ++l) v += g.n[l][s] * sm.tl[l * D3 + j];
      sm.r[idx] = v;
      sm.x[idx] = v;
    }
    __syncthreads();
    spd_apply<D3, TILE>(sm.L, sm.x, sm.tmp, 3);  // x_s = M^{-1} r_s
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
    spd_apply<D3, TILE>(sm.LS, sm.u, sm.tmp, 1);  // u = S^{-1} rhs_u
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
    spd_apply<D3, TILE>(sm.L, sm.x, sm.tmp, 3);  // q_s = M^{-1} x_s
    for (int idx = t; idx < 3 * D3; idx += nt) qout[(size_t)E * 3 * D3 + idx] = sm.x[idx];
    for (int i = t; i < D3; i += nt) uout[(size_t)E * D3 + i] = sm.u[i];
    __syncthreads();
  }
}

// ---- degrees 1..3: four elements per wavefront on the FP64 matrix cores, with the tile
// factor store of the condensation (U^{-1} and Us^{-1} as packed upper 4x4 tiles, f as
// tiles with the values in column 0).  Vectors are tiles whose four columns are equal.
// With mfma4(A, B) = A^T B:
//   U^T v:  (U^T v)(K) = sum_{J<=K} mfma4(U(J,K), v(J))
//   U v:    (U v)(J)   = sum_{K>=J} mfma4(U(J,K)^T, v(K))   (tiles transposed once)
template <int K>
struct RD {
  static constexpr int D3 = dim3(K), D2 = dim2(K), T = (D3 + 3) / 4, JT = (D2 + 3) / 4;
  static constexpr int NU = T * (T + 1) / 2, D3P4 = 4 * T, D2P4 = 4 * JT;
  // factor store of the tile condensation: U^{-1}, Us^{-1}, f, then the geometry record
  static constexpr int GEO_OFF = (2 * NU + T) * 16, FLEN = GEO_OFF + kGeoRecord;
};

template <int T>
__device__ __forceinline__ void apply_Ut(const double (&U)[T * (T + 1) / 2], const double (&v)[T], double (&y)[T]) {
#pragma unroll
  for (int Kt = 0; Kt < T; ++Kt) {
    double acc = 0.0;
#pragma unroll
    for (int J = 0; J <= Kt; ++J) acc = mfma4(U[utile(J, Kt, T)], v[J], acc);
    y[Kt] = acc;
  }
}

template <int T>
__device__ __forceinline__ void apply_U(const double (&UT)[T * (T + 1) / 2], const double (&y)[T], double (&x)[T]) {
#pragma unroll
  for (int J = 0; J < T; ++J) {
    double acc = 0.0;
#pragma unroll
    for (int Kt = J; Kt < T; ++Kt) acc = mfma4(UT[utile(J, Kt, T)], y[Kt], acc);
    x[J] = acc;
  }
}

constexpr int kRecWaves = 4;

template <int K>
__global__ void __launch_bounds__(64 * kRecWaves, 2) k_recover_tile(hdg_mesh mesh, Tables tb,
                                                                 const double* __restrict__ tau,
                                                                 const double* __restrict__ factors,
                                                                 const double* __restrict__ uhat,
                                                                 double* __restrict__ qout,
                                                                 double* __restrict__ uout) {
  using D = RD<K>;
  constexpr int D3 = D::D3, D2 = D::D2, T = D::T, JT = D::JT, NU = D::NU, D3P4 = D::D3P4, D2P4 = D::D2P4;
  constexpr int L3 = D3P4 * D3P4, LDP = 24 * D3P4 * D2P4;
  // the DP and Chat tables, shared by the workgroup's wavefronts, copied global->LDS
  // asynchronously (1 KB per instruction, spread over the wavefronts)
  __shared__ __attribute__((aligned(16))) double s_dpt[lds_stage_bytes<LDP>() / 8];
  __shared__ __attribute__((aligned(16))) double s_cht[lds_stage_bytes<3 * L3>() / 8];
  lds_stage_wg<LDP, kRecWaves>(tb.DPT, s_dpt, threadIdx.x >> 6, threadIdx.x & 63);
  lds_stage_wg<3 * L3, kRecWaves>(tb.ChatT, s_cht, threadIdx.x >> 6, threadIdx.x & 63);
  lds_stage_wait();
  __syncthreads();
  // per-wavefront geometry records and face numbers (each wavefront runs its own loop, so
  // only the wavefront syncs)
  __shared__ double s_geo_[kRecWaves][4][kGeoRecord];
  __shared__ int s_fbe_[kRecWaves][4][4];
  const int wave = threadIdx.x >> 6;
  auto& s_geo = s_geo_[wave];
  auto& s_fbe = s_fbe_[wave];
  const int ngroups = (mesh.nelt + 3) / 4;
  for (int grp = blockIdx.x * kRecWaves + wave; grp < ngroups; grp += gridDim.x * kRecWaves) {
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int r = (lane >> 4) & 3, c = lane & 3, blk = (lane >> 2) & 3;
    wave_lds_sync();
    {
      // the geometry records, kept in the factor store by the condensation, and the face
      // numbers: every load of the group is issued before any is used (indices clamped;
      // padding slots of a ragged last group get zeros)
      constexpr int GIT = 4 * kGeoRecord / 64;
      static_assert(4 * kGeoRecord % 64 == 0, "geometry records in whole passes");
      double gv[GIT];
#pragma unroll
      for (int j = 0; j < GIT; ++j) {
        const int idx = lane + 64 * j, Ee = 4 * grp + idx / kGeoRecord;
        gv[j] = factors[(Ee < mesh.nelt ? (size_t)Ee * D::FLEN : 0) + D::GEO_OFF + idx % kGeoRecord];
      }
      const int ef = 4 * grp + ((lane >> 2) & 3);
      const int fb = mesh.d_facebyele[4 * (size_t)(ef < mesh.nelt ? ef : 0) + (lane & 3)];
#pragma unroll
      for (int j = 0; j < GIT; ++j) {
        const int idx = lane + 64 * j;
        (&s_geo[0][0])[idx] = 4 * grp + idx / kGeoRecord < mesh.nelt ? gv[j] : 0.0;
      }
      if (lane < 16) s_fbe[lane >> 2][lane & 3] = ef < mesh.nelt ? fb : 0;
    }
    wave_lds_sync();
    const int E = 4 * grp + blk < mesh.nelt ? 4 * grp + blk : -1;
    const double* geo = s_geo[blk];
    const double* fa = factors + (size_t)(E >= 0 ? E : 0) * D::FLEN;  // padding lanes read element 0
    double Ui[NU], UiT[NU];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      Ui[i] = fa[i * 16 + 4 * r + c];
      UiT[i] = tile_transpose(Ui[i]);
    }
    // t_l = DP_l^T uhat_l, folded into r_s = sum_l n_ls t_l and rhs = f + sum_l T_l t_l
    double rs[3][T], ru[T];
#pragma unroll
    for (int Kt = 0; Kt < T; ++Kt) {
      ru[Kt] = fa[(2 * NU + Kt) * 16 + 4 * r];  // f (column 0 of its tile)
      rs[0][Kt] = rs[1][Kt] = rs[2][Kt] = 0.0;
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int fbe = s_fbe[blk][l];
      const double* dpt = s_dpt + ((int)geo[G_MU + l] * 4 + l) * D3P4 * D2P4;
      double uh[JT];
#pragma unroll
      for (int J = 0; J < JT; ++J) {
        const int i = 4 * J + r;
        uh[J] = (E >= 0 && i < D2) ? uhat[(size_t)fbe * D2 + i] : 0.0;
      }
      const double n0 = geo[G_N + 3 * l], n1 = geo[G_N + 3 * l + 1], n2 = geo[G_N + 3 * l + 2], Tl = geo[G_T + l];
#pragma unroll
      for (int Kt = 0; Kt < T; ++Kt) {
        double t = 0.0;
#pragma unroll
        for (int J = 0; J < JT; ++J) t = mfma4(dpt[(4 * Kt + c) * D2P4 + 4 * J + r], uh[J], t);
        rs[0][Kt] += n0 * t;
        rs[1][Kt] += n1 * t;
        rs[2][Kt] += n2 * t;
        ru[Kt] += Tl * t;
      }
    }
    const double* a = geo + G_A;
    // x_s = M^{-1} r_s, v_h = sum_s a_sh x_s, rhs += sum_h Chat^h v_h
    {
      double xs[3][T];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        double y[T];
        apply_Ut<T>(Ui, rs[s], y);
        apply_U<T>(UiT, y, xs[s]);
      }
#pragma unroll
      for (int h = 0; h < 3; ++h) {
        double v[T];
#pragma unroll
        for (int J = 0; J < T; ++J) v[J] = a[h] * xs[0][J] + a[3 + h] * xs[1][J] + a[6 + h] * xs[2][J];
#pragma unroll
        for (int Kt = 0; Kt < T; ++Kt) {
          double acc = ru[Kt];
#pragma unroll
          for (int J = 0; J < T; ++J) acc = mfma4(s_cht[h * L3 + (4 * J + r) * D3P4 + 4 * Kt + c], v[J], acc);
          ru[Kt] = acc;
        }
      }
    }
    // u = S^{-1} rhs with the factors of S.  The hybridized BDM element (record slot G_DU:
    // d2 removed modes) has u in P_{k-1}: the removed rows of the right-hand side are dropped,
    // and S^{-1} is the identity there, so those modes of u come out zero.
    {
      const int d3u = D3 - (int)geo[G_DU];
#pragma unroll
      for (int Kt = 0; Kt < T; ++Kt) ru[Kt] = 4 * Kt + r < d3u ? ru[Kt] : 0.0;
    }
    double uu[T];
    {
#pragma unroll
      for (int i = 0; i < NU; ++i) {
        Ui[i] = fa[(NU + i) * 16 + 4 * r + c];
        UiT[i] = tile_transpose(Ui[i]);
      }
      double y[T];
      apply_Ut<T>(Ui, ru, y);
      apply_U<T>(UiT, y, uu);
#pragma unroll
      for (int i = 0; i < NU; ++i) {  // back to the factors of M
        Ui[i] = fa[i * 16 + 4 * r + c];
        UiT[i] = tile_transpose(Ui[i]);
      }
    }
    // x_s = C_s^T u - r_s = sum_h a_sh Chat^{hT} u - r_s, q_s = M^{-1} x_s
    double w[3][T];
#pragma unroll
    for (int h = 0; h < 3; ++h)
#pragma unroll
      for (int Kt = 0; Kt < T; ++Kt) {
        double acc = 0.0;
#pragma unroll
        for (int J = 0; J < T; ++J) acc = mfma4(s_cht[h * L3 + (4 * Kt + c) * D3P4 + 4 * J + r], uu[J], acc);
        w[h][Kt] = acc;
      }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      double x[T], y[T], qs[T];
#pragma unroll
      for (int Kt = 0; Kt < T; ++Kt) x[Kt] = a[3 * s] * w[0][Kt] + a[3 * s + 1] * w[1][Kt] + a[3 * s + 2] * w[2][Kt] - rs[s][Kt];
      apply_Ut<T>(Ui, x, y);
      apply_U<T>(UiT, y, qs);
      if (E >= 0 && c == 0) {
#pragma unroll
        for (int Kt = 0; Kt < T; ++Kt) {
          const int i = 4 * Kt + r;
          if (i < D3) qout[((size_t)E * 3 + s) * D3 + i] = qs[Kt];
        }
      }
    }
    if (E >= 0 && c == 0) {
#pragma unroll
      for (int Kt = 0; Kt < T; ++Kt) {
        const int i = 4 * Kt + r;
        if (i < D3) uout[(size_t)E * D3 + i] = uu[Kt];
      }
    }
  }
}

template <int K>
hdg_status run_recover(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* tau,
                       const double* factors, const double* uhat, double* q, double* u, double* us, hipStream_t s) {
  if constexpr (K >= 1 && K <= 3) {
    const int64_t groups = (mesh->nelt + 3) / 4;
    const int64_t wgs = (groups + kRecWaves - 1) / kRecWaves;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(wgs, 2 * (int64_t)device_cu_count()));
    timer_begin("k_recover_tile", s);
    k_recover_tile<K><<<grid, 64 * kRecWaves, 0, s>>>(*mesh, disc->dev, tau, factors, uhat, q, u);
    timer_end("k_recover_tile", s);
  } else {
    const int grid = (int)std::min<int64_t>(mesh->nelt, 1 << 20);
    timer_begin("k_recover", s);
    k_recover<K, false><<<grid, recover_threads(K), 0, s>>>(*mesh, disc->dev, kappa, tau, factors, uhat, q, u);
    timer_end("k_recover", s);
  }
  HDG_CHECK_LAUNCH("k_recover");
  return us ? launch_postprocess(disc, mesh, kappa, tau, q, u, factors, us, s) : HDG_OK;
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
    case 5: return run_recover<5>(disc, mesh, d_kappa, d_tau, d_factors, d_uhat, d_q, d_u, d_ustar, s);
    case 6: return run_recover<6>(disc, mesh, d_kappa, d_tau, d_factors, d_uhat, d_q, d_u, d_ustar, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_recover: unsupported degree");
}
