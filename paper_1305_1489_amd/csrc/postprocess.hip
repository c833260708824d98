// Local postprocess u* of degree k+1 (eq 9.11) on the FP64 matrix cores, four elements
// per wavefront.
//
// For each element, with q_h = sum_j Q_s[j] P_j (the recovered flux) and u_h:
//   S*_{ij} = int_K grad P_i . grad P_j = sum_{h<=g} G_{hg} Shat^{hg}_{ij},  G = a^T a / det,
//   rhs_i   = -int_K kappa^{-1} q_h . grad P_i
//           = -sum_h sum_q Y_h(q) gradhat_h P_i(p_q),
//   Y_h(q)  = |K| w_q kappa(x_q)^{-1} / det * sum_j P_j(p_q) V[j][h],   V = Q a,
// where a = det(B) B^{-T} is the cofactor matrix of the element map.  The basis is
// orthonormal and hierarchical, so the mean condition of eq 9.11 reads u*_0 = u_0, and the
// gradient rows of mode 0 vanish: S* is set to the identity on mode 0 (and on the padding
// modes), rhs_0 = u_0, and one SPD solve gives every coefficient.
//
// Layouts.  The right-hand side is a contraction over the 3 x nqd (direction, point)
// pairs with a single right-hand side per element; putting one element per matrix-core
// block would leave three of the four columns of every product idle.  It is computed
// split-K instead: the tile columns are the four elements of the group and the four
// blocks take interleaved chunks of the quadrature points; a cross-block sum finishes it.
// The stiffness matrix, its blocked Cholesky and the two triangular solves use the
// element-per-block layout of the condensation kernels (vectors as tiles whose four
// columns are equal).
#include "tile.h"

namespace hdg {
namespace {

template <int K>
struct PD {
  static constexpr int D3 = dim3(K);
  static constexpr int D3P = dim3(K + 1);
  static constexpr int NQD = (K + 2) * (K + 2) * (K + 2);
  static constexpr int NQP = (NQD + 3) / 4 * 4;
  static constexpr int QT = NQP / 4;         // point tiles
  static constexpr int QI = (QT + 3) / 4;    // point tiles per block
  static constexpr int D3P4 = (D3 + 3) / 4 * 4;
  static constexpr int JT = D3P4 / 4;        // tiles of the degree-k modes
  static constexpr int TS = (D3P + 3) / 4;   // tiles of the degree-(k+1) modes
  static constexpr int NUS = TS * (TS + 1) / 2;
};

enum { PG_A = 0, PG_DET = 9, PG_VOL = 10, PG_LEN = 11 };

__device__ __forceinline__ double lane_read(double v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

template <int K>
__global__ void __launch_bounds__(64) k_postprocess(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                    const double* __restrict__ tau, const double* __restrict__ qin,
                                                    const double* __restrict__ uin, double* __restrict__ usout) {
  using D = PD<K>;
  constexpr int D3 = D::D3, D3P = D::D3P, NQD = D::NQD, NQP = D::NQP, QT = D::QT, QI = D::QI;
  constexpr int D3P4 = D::D3P4, JT = D::JT, TS = D::TS, NUS = D::NUS, D3PP4 = 4 * TS;
  __shared__ double s_geo[4][PG_LEN];
  __shared__ int s_E[4];
  __shared__ double s_x[64];
  const int ngroups = (mesh.nelt + 3) / 4;
  for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    // per-group opaque lane index: keeps the table addresses derived from it inside the
    // loop (hoisted, they would outlive the register file)
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    const int r = lane >> 4, c = lane & 3, blk = (lane >> 2) & 3;
    __syncthreads();
    if (lane < 4) {
      const int E = 4 * grp + lane < mesh.nelt ? 4 * grp + lane : -1;
      s_E[lane] = E;
      ElemGeom g;
      if (E >= 0) {
        load_geometry(E, mesh, tau, g);
      } else {  // padding element: reference geometry, zero data, outputs not written
        g = ElemGeom{};
        g.a[0][0] = g.a[1][1] = g.a[2][2] = 1.0;
        g.det = 1.0;
        g.vol = 1.0 / 6.0;
      }
      for (int i = 0; i < 9; ++i) s_geo[lane][PG_A + i] = g.a[i / 3][i % 3];
      s_geo[lane][PG_DET] = g.det;
      s_geo[lane][PG_VOL] = g.vol;
    }
    __syncthreads();

    // ---- V = Q a, elements in the tile columns: lane (r, c) of tile J holds V_c[4J + r][h]
    double V[3][JT];
    {
      const int E = s_E[c];
      const double* a = s_geo[c] + PG_A;
#pragma unroll
      for (int J = 0; J < JT; ++J) {
        const int j = 4 * J + r;
        double qs[3] = {0.0, 0.0, 0.0};
        if (E >= 0 && j < D3) {
#pragma unroll
          for (int s = 0; s < 3; ++s) qs[s] = qin[((size_t)E * 3 + s) * D3 + j];
        }
#pragma unroll
        for (int h = 0; h < 3; ++h) V[h][J] = qs[0] * a[h] + qs[1] * a[3 + h] + qs[2] * a[6 + h];
      }
    }

    // ---- rhs, split-K over the points: block blk takes point tiles blk, blk + 4, ...
    double R[TS];
#pragma unroll
    for (int I = 0; I < TS; ++I) R[I] = 0.0;
    {
      const int E = s_E[c];
      const double wscale = s_geo[c][PG_VOL] / s_geo[c][PG_DET];
#pragma unroll 1
      for (int qi = 0; qi < QI; ++qi) {
        const int Qt = 4 * qi + blk;
        const int Ql = Qt < QT ? Qt : QT - 1;  // tiles past the end load in bounds, weigh zero
        // Y_h tile: rows = points 4Qt + r, columns = elements
        double xp[JT];
#pragma unroll
        for (int J = 0; J < JT; ++J) xp[J] = tb.Pt[(4 * Ql + c) * D3P4 + 4 * J + r];
        const int q = 4 * Qt + r;
        double wr = 0.0;
        if (Qt < QT && q < NQD && E >= 0) wr = wscale * tb.vol_w[q] / kappa[(size_t)E * NQD + q];
        double y[3];
#pragma unroll
        for (int h = 0; h < 3; ++h) {
          double acc = 0.0;
#pragma unroll
          for (int J = 0; J < JT; ++J) acc = mfma4(xp[J], V[h][J], acc);
          y[h] = wr * acc;
        }
#pragma unroll
        for (int h = 0; h < 3; ++h) {
          const double* g = tb.P1gt + ((size_t)h * NQP + 4 * Ql + r) * D3PP4 + c;
#pragma unroll
          for (int I = 0; I < TS; ++I) R[I] = mfma4(g[4 * I], y[h], R[I]);
        }
      }
    }
    // sum over the four point chunks (identical, order-independent result in every block),
    // then to the element-per-block layout: lane (r, blk, c) takes R[r][blk]
    double rhs[TS];
#pragma unroll
    for (int I = 0; I < TS; ++I) {
      double v = R[I];
      v += lane_read(v, lane ^ 4);
      v += lane_read(v, lane ^ 8);
      rhs[I] = -lane_read(v, (lane & 0x3c) | blk);
    }
    const int Eb = s_E[blk];
    if (r == 0) rhs[0] = Eb >= 0 ? uin[(size_t)Eb * D3] : 0.0;  // mean condition: u*_0 = u_0

    // ---- S* = sum_p cf_p Shat_p on the upper tiles, identity on mode 0 and the padding
    double S[NUS];
    {
      const double* a = s_geo[blk] + PG_A;
      const double idet = 1.0 / s_geo[blk][PG_DET];
      double G[3][3];
#pragma unroll
      for (int h = 0; h < 3; ++h)
#pragma unroll
        for (int k = 0; k < 3; ++k) G[h][k] = (a[h] * a[k] + a[3 + h] * a[3 + k] + a[6 + h] * a[6 + k]) * idet;
      const double cf[6] = {G[0][0], G[1][1], G[2][2], G[0][1], G[0][2], G[1][2]};
#pragma unroll
      for (int I = 0; I < TS; ++I)
#pragma unroll
        for (int N = I; N < TS; ++N) {
          const int u = utile(I, N, TS);
          double s = 0.0;
#pragma unroll
          for (int p = 0; p < 6; ++p) s += cf[p] * tb.Shatt[(p * NUS + u) * 16 + 4 * r + c];
          const int i = 4 * I + r, j = 4 * N + c;
          if (i == 0 || j == 0 || i >= D3P || j >= D3P) s = (i == j) ? 1.0 : 0.0;
          S[u] = s;
        }
    }
    __builtin_amdgcn_sched_barrier(0);

    // ---- S* = U^T U, then U^T y = rhs, U x = y
    double Vd[TS];
    tile_cholesky<TS>(S, Vd, s_x);
    double x[TS];
#pragma unroll
    for (int I = 0; I < TS; ++I) {
      double t = 0.0;
#pragma unroll
      for (int J = 0; J < I; ++J) t = mfma4(S[utile(J, I, TS)], x[J], t);
      x[I] = mfma4(Vd[I], rhs[I] - t, 0.0);
    }
#pragma unroll
    for (int I = TS - 1; I >= 0; --I) {
      double t = 0.0;
#pragma unroll
      for (int N = I + 1; N < TS; ++N) t = mfma4(tile_transpose(S[utile(I, N, TS)]), x[N], t);
      x[I] = mfma4(tile_transpose(Vd[I]), x[I] - t, 0.0);
    }
    if (Eb >= 0 && c == 0) {
#pragma unroll
      for (int I = 0; I < TS; ++I) {
        const int i = 4 * I + r;
        if (i < D3P) usout[(size_t)Eb * D3P + i] = x[I];
      }
    }
  }
}

}  // namespace

// Launches the postprocess for degree k on every element of the mesh; q and u are the
// recovered fields (layouts of hdg_recover).
hdg_status launch_postprocess(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* tau,
                              const double* q, const double* u, double* us, hipStream_t s) {
  const int64_t groups = (mesh->nelt + 3) / 4;
  if (groups == 0) return HDG_OK;
  const int grid = (int)std::min<int64_t>(groups, 1 << 20);
  switch (disc->host.k) {
    case 0: k_postprocess<0><<<grid, 64, 0, s>>>(*mesh, disc->dev, kappa, tau, q, u, us); break;
    case 1: k_postprocess<1><<<grid, 64, 0, s>>>(*mesh, disc->dev, kappa, tau, q, u, us); break;
    case 2: k_postprocess<2><<<grid, 64, 0, s>>>(*mesh, disc->dev, kappa, tau, q, u, us); break;
    case 3: k_postprocess<3><<<grid, 64, 0, s>>>(*mesh, disc->dev, kappa, tau, q, u, us); break;
    case 4: k_postprocess<4><<<grid, 64, 0, s>>>(*mesh, disc->dev, kappa, tau, q, u, us); break;
    default: return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_recover: unsupported degree");
  }
  HDG_CHECK_LAUNCH("k_postprocess");
  return HDG_OK;
}

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who);

}  // namespace hdg

extern "C" hdg_status hdg_postprocess(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                      const double* d_tau, const double* d_q, const double* d_u, double* d_ustar,
                                      void* stream) {
  hdg_status st = hdg::check_disc_mesh(disc, mesh, "hdg_postprocess");
  if (st) return st;
  if (!d_kappa || !d_tau || !d_q || !d_u || !d_ustar)
    return hdg::set_error(HDG_ERR_INVALID_ARG, "hdg_postprocess: NULL array");
  return hdg::launch_postprocess(disc, mesh, d_kappa, d_tau, d_q, d_u, d_ustar, (hipStream_t)stream);
}
