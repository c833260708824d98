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
// Two kernels, each keeping the tables it streams resident in LDS and shared by the
// wavefronts of a workgroup (each wavefront runs its own persistent loop over groups of
// four elements):
//   k_pp_rhs    the right-hand side, into the u* array (gradient tables: 131 KB at k = 3).
//               The contraction over the 3 x nqd (direction, point) pairs has a single
//               right-hand side per element; one element per matrix-core block would leave
//               three of the four columns of every product idle.  It runs split-K instead:
//               the tile columns are the four elements of the group, the four blocks take
//               interleaved chunks of the quadrature points, and a cross-block sum
//               finishes it.
//   k_pp_solve  S* from the six stiffness tables (LDS), blocked Cholesky, the two
//               triangular solves, in the element-per-block layout of the condensation
//               kernels (vectors as tiles whose four columns are equal).
// Geometry is computed by lanes 0..3 (one element each) and shared by lane permutes.
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
  static constexpr int D3PP4 = 4 * TS;
  static constexpr int P1_LEN = 3 * NQP * D3PP4, PT_LEN = NQP * D3P4, SH_LEN = 6 * NUS * 16;
  // LDS copies: row strides padded by one double, so that the four blocks' point tiles
  // (4 rows apart) start in different banks
  static constexpr int P1_LD = D3PP4 + 1, PT_LD = D3P4 + 1;
  static constexpr int P1_LDS_LEN = 3 * NQP * P1_LD, PT_LDS_LEN = NQP * PT_LD;
  // the gradient tables stay in global memory when they do not fit next to each other in LDS
  static constexpr bool RHS_LDS = (P1_LDS_LEN + PT_LDS_LEN) * 8 <= 144 * 1024;
};

constexpr int kRhsWaves = 16, kSolveWaves = 4;

// Geometry of element E (lanes 0..3; E < 0: the reference element, data zero).
struct PGeo {
  double a[9], det, vol;
};

__device__ __forceinline__ PGeo pp_geometry(int E, const hdg_mesh& mesh, const double* tau) {
  PGeo p{};
  if (E >= 0) {
    ElemGeom g;
    load_geometry(E, mesh, tau, g);
    for (int i = 0; i < 9; ++i) p.a[i] = g.a[i / 3][i % 3];
    p.det = g.det;
    p.vol = g.vol;
  } else {
    p.a[0] = p.a[4] = p.a[8] = 1.0;
    p.det = 1.0;
    p.vol = 1.0 / 6.0;
  }
  return p;
}

// Geometry of element E from the record the tile condensation keeps in its factor store
// (fac: that store, degrees 1..3), else computed; the same bits either way.
template <int K>
__device__ __forceinline__ PGeo pp_geometry_any(int E, const hdg_mesh& mesh, const double* tau,
                                                const double* __restrict__ fac) {
  if (!fac || E < 0) return pp_geometry(E, mesh, tau);
  constexpr int T = (dim3(K) + 3) / 4, NU = T * (T + 1) / 2, GEO_OFF = (2 * NU + T) * 16;
  const double* rec = fac + (size_t)E * (GEO_OFF + kGeoRecord) + GEO_OFF;
  PGeo p;
  for (int i = 0; i < 9; ++i) p.a[i] = rec[G_A + i];
  p.det = rec[G_DET];
  p.vol = rec[G_VOL];
  return p;
}

template <int K>
__global__ void __launch_bounds__(64 * kRhsWaves) k_pp_rhs(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                           const double* __restrict__ tau,
                                                           const double* __restrict__ fac,
                                                           const double* __restrict__ qin,
                                                           const double* __restrict__ uin,
                                                           double* __restrict__ rhs_out) {
  using D = PD<K>;
  constexpr int D3 = D::D3, D3P = D::D3P, NQD = D::NQD, NQP = D::NQP, QT = D::QT, QI = D::QI;
  constexpr int D3P4 = D::D3P4, JT = D::JT, TS = D::TS, D3PP4 = D::D3PP4;
  __shared__ double s_p1t[D::RHS_LDS ? D::P1_LDS_LEN : 1];
  __shared__ double s_ptt[D::RHS_LDS ? D::PT_LDS_LEN : 1];
  if constexpr (D::RHS_LDS) {
    for (int i = threadIdx.x; i < D::P1_LEN; i += blockDim.x) s_p1t[(i / D3PP4) * D::P1_LD + i % D3PP4] = tb.P1gt[i];
    for (int i = threadIdx.x; i < D::PT_LEN; i += blockDim.x) s_ptt[(i / D3P4) * D::PT_LD + i % D3P4] = tb.Pt[i];
    __syncthreads();
  }
  const double* s_p1 = D::RHS_LDS ? s_p1t : tb.P1gt;
  const double* s_pt = D::RHS_LDS ? s_ptt : tb.Pt;
  constexpr int P1S = D::RHS_LDS ? D::P1_LD : D3PP4, PTS = D::RHS_LDS ? D::PT_LD : D3P4;
  const int ngroups = (mesh.nelt + 3) / 4;
  const int wave = threadIdx.x >> 6;
  for (int grp = blockIdx.x * kRhsWaves + wave; grp < ngroups; grp += gridDim.x * kRhsWaves) {
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int r = lane >> 4, c = lane & 3, blk = (lane >> 2) & 3;
    const int Em = 4 * grp + (lane & 3);
    const int Eown = Em < mesh.nelt ? Em : -1;
    PGeo gl{};
    if (lane < 4) gl = pp_geometry_any<K>(Eown, mesh, tau, fac);
    // element c's geometry (lane c computed it)
    double a[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) a[i] = lane_read(gl.a[i], c);
    const double wscale = lane_read(gl.vol, c) / lane_read(gl.det, c);
    const int Ec = 4 * grp + c < mesh.nelt ? 4 * grp + c : -1;

    // ---- V = Q a, elements in the tile columns: lane (r, c) of tile J holds V_c[4J + r][h]
    // every global load of the group is issued before any is used (indices clamped instead
    // of branched around), so that their latencies overlap
    constexpr bool PRE = QI <= 8;  // the point coefficients too, while registers allow
    double qv[JT][3], kap[PRE ? QI : 1], vw[PRE ? QI : 1];
#pragma unroll
    for (int J = 0; J < JT; ++J) {
      const int j = 4 * J + r;
      const size_t o = (Ec >= 0 && j < D3) ? (size_t)Ec * 3 * D3 + j : 0;
#pragma unroll
      for (int s = 0; s < 3; ++s) qv[J][s] = qin[o + (size_t)s * D3];
    }
#pragma unroll
    for (int qi = 0; qi < (PRE ? QI : 0); ++qi) {
      const int Qt = 4 * qi + blk, q = 4 * Qt + r;
      const bool ok = Qt < QT && q < NQD && Ec >= 0;
      kap[qi] = kappa[ok ? (size_t)Ec * NQD + q : 0];
      vw[qi] = tb.vol_w[ok ? q : 0];
    }
    double V[3][JT];
#pragma unroll
    for (int J = 0; J < JT; ++J) {
      const bool ok = Ec >= 0 && 4 * J + r < D3;
      const double q0 = ok ? qv[J][0] : 0.0, q1 = ok ? qv[J][1] : 0.0, q2 = ok ? qv[J][2] : 0.0;
#pragma unroll
      for (int h = 0; h < 3; ++h) V[h][J] = q0 * a[h] + q1 * a[3 + h] + q2 * a[6 + h];
    }
    // ---- split-K over the points: block blk takes point tiles blk, blk + 4, ...
    double R[TS];
#pragma unroll
    for (int I = 0; I < TS; ++I) R[I] = 0.0;
#pragma unroll(PRE ? QI : 2)
    for (int qi = 0; qi < QI; ++qi) {
      const int Qt = 4 * qi + blk;
      const int Ql = Qt < QT ? Qt : QT - 1;  // tiles past the end read in bounds, weigh zero
      double xp[JT];
#pragma unroll
      for (int J = 0; J < JT; ++J) xp[J] = s_pt[(4 * Ql + c) * PTS + 4 * J + r];
      const int q = 4 * Qt + r;
      double wr = 0.0;
      if constexpr (PRE) {
        wr = (Qt < QT && q < NQD && Ec >= 0) ? wscale * vw[qi] / kap[qi] : 0.0;
      } else {
        if (Qt < QT && q < NQD && Ec >= 0) wr = wscale * tb.vol_w[q] / kappa[(size_t)Ec * NQD + q];
      }
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
        const double* g = s_p1 + (h * NQP + 4 * Ql + r) * P1S + c;
#pragma unroll
        for (int I = 0; I < TS; ++I) R[I] = mfma4(g[4 * I], y[h], R[I]);
      }
    }
    // sum over the four point chunks (every block gets the same value, whatever the
    // order), then lane (r, blk, 0) stores mode 4I + r of element blk
    const int Eb = 4 * grp + blk < mesh.nelt ? 4 * grp + blk : -1;
#pragma unroll
    for (int I = 0; I < TS; ++I) {
      double v = R[I];
      v += lane_read(v, lane ^ 4);
      v += lane_read(v, lane ^ 8);
      v = -lane_read(v, (lane & 0x3c) | blk);
      const int i = 4 * I + r;
      if (i == 0) v = Eb >= 0 ? uin[(size_t)Eb * D3] : 0.0;  // mean condition: u*_0 = u_0
      if (Eb >= 0 && c == 0 && i < D3P) rhs_out[(size_t)Eb * D3P + i] = v;
    }
  }
}

template <int K>
__global__ void __launch_bounds__(64 * kSolveWaves, 2) k_pp_solve(hdg_mesh mesh, Tables tb,
                                                               const double* __restrict__ tau,
                                                               const double* __restrict__ fac,
                                                               double* __restrict__ us) {
  using D = PD<K>;
  constexpr int D3P = D::D3P, TS = D::TS, NUS = D::NUS;
  __shared__ double s_sh[D::SH_LEN];
  __shared__ double s_x[kSolveWaves][64];
  for (int i = threadIdx.x; i < D::SH_LEN; i += blockDim.x) s_sh[i] = tb.Shatt[i];
  __syncthreads();
  const int ngroups = (mesh.nelt + 3) / 4;
  const int wave = threadIdx.x >> 6;
  double* xch = s_x[wave];
  for (int grp = blockIdx.x * kSolveWaves + wave; grp < ngroups; grp += gridDim.x * kSolveWaves) {
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int r = lane >> 4, c = lane & 3, blk = (lane >> 2) & 3;
    const int Em = 4 * grp + (lane & 3);
    PGeo gl{};
    if (lane < 4) gl = pp_geometry_any<K>(Em < mesh.nelt ? Em : -1, mesh, tau, fac);
    const int Eb = 4 * grp + blk < mesh.nelt ? 4 * grp + blk : -1;
    // ---- S* = sum_p cf_p Shat_p on the upper tiles, identity on mode 0 and the padding
    double S[NUS];
    {
      double a[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) a[i] = lane_read(gl.a[i], blk);
      const double idet = 1.0 / lane_read(gl.det, blk);
      double G[3][3];
#pragma unroll
      for (int h = 0; h < 3; ++h)
#pragma unroll
        for (int k = 0; k < 3; ++k) G[h][k] = (a[h] * a[k] + a[3 + h] * a[3 + k] + a[6 + h] * a[6 + k]) * idet;
      const double cf[6] = {G[0][0], G[1][1], G[2][2], G[0][1], G[0][2], G[1][2]};
#pragma unroll
      for (int I = 0; I < TS; ++I) {
#pragma unroll
        for (int N = I; N < TS; ++N) {
          const int u = utile(I, N, TS);
          double s = 0.0;
#pragma unroll
          for (int p = 0; p < 6; ++p) s += cf[p] * s_sh[(p * NUS + u) * 16 + 4 * r + c];
          const int i = 4 * I + r, j = 4 * N + c;
          if (i == 0 || j == 0 || i >= D3P || j >= D3P) s = (i == j) ? 1.0 : 0.0;
          S[u] = s;
        }
        __builtin_amdgcn_sched_barrier(0);  // one tile row of table reads in flight at a time
      }
    }
    // ---- S* = U^T U, then U^T y = rhs, U x = y
    double Vd[TS];
    tile_cholesky<TS, true>(S, Vd, xch);
    // right-hand side (written by k_pp_rhs into the u* array), column-replicated tiles
    double rhs[TS];
#pragma unroll
    for (int I = 0; I < TS; ++I) {
      const int i = 4 * I + r;
      rhs[I] = (Eb >= 0 && i < D3P) ? us[(size_t)Eb * D3P + i] : 0.0;
    }
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
        if (i < D3P) us[(size_t)Eb * D3P + i] = x[I];
      }
    }
  }
}

template <int K>
hdg_status run_postprocess(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* tau,
                           const double* q, const double* u, const double* factors, double* us, hipStream_t s) {
  const double* fac = (K >= 1 && K <= 3) ? factors : nullptr;  // only the tile layouts carry the record
  const int64_t groups = (mesh->nelt + 3) / 4;
  const int ncu = device_cu_count();
  const int g1 = (int)std::max<int64_t>(1, std::min<int64_t>((groups + kRhsWaves - 1) / kRhsWaves, ncu));
  timer_begin("k_pp_rhs", s);
  k_pp_rhs<K><<<g1, 64 * kRhsWaves, 0, s>>>(*mesh, disc->dev, kappa, tau, fac, q, u, us);
  timer_end("k_pp_rhs", s);
  const int g2 = (int)std::max<int64_t>(1, std::min<int64_t>((groups + kSolveWaves - 1) / kSolveWaves, 3 * ncu));
  timer_begin("k_pp_solve", s);
  k_pp_solve<K><<<g2, 64 * kSolveWaves, 0, s>>>(*mesh, disc->dev, tau, fac, us);
  timer_end("k_pp_solve", s);
  HDG_CHECK_LAUNCH("k_pp_rhs / k_pp_solve");
  return HDG_OK;
}

}  // namespace

// Launches the postprocess for degree k on every element of the mesh; q and u are the
// recovered fields (layouts of hdg_recover).  us doubles as the right-hand side between
// the two kernels.
hdg_status launch_postprocess(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* tau,
                              const double* q, const double* u, const double* factors, double* us, hipStream_t s) {
  if (mesh->nelt == 0) return HDG_OK;
  switch (disc->host.k) {
    case 0: return run_postprocess<0>(disc, mesh, kappa, tau, q, u, factors, us, s);
    case 1: return run_postprocess<1>(disc, mesh, kappa, tau, q, u, factors, us, s);
    case 2: return run_postprocess<2>(disc, mesh, kappa, tau, q, u, factors, us, s);
    case 3: return run_postprocess<3>(disc, mesh, kappa, tau, q, u, factors, us, s);
    case 4: return run_postprocess<4>(disc, mesh, kappa, tau, q, u, factors, us, s);
    case 5:
    case 6: return launch_postprocess_big(disc, mesh, kappa, tau, q, u, us, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_recover: unsupported degree");
}

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who);

}  // namespace hdg

extern "C" hdg_status hdg_postprocess(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                      const double* d_tau, const double* d_q, const double* d_u,
                                      const double* d_factors, double* d_ustar, void* stream) {
  hdg_status st = hdg::check_disc_mesh(disc, mesh, "hdg_postprocess");
  if (st) return st;
  if (!d_kappa || !d_tau || !d_q || !d_u || !d_ustar)
    return hdg::set_error(HDG_ERR_INVALID_ARG, "hdg_postprocess: NULL array");
  return hdg::launch_postprocess(disc, mesh, d_kappa, d_tau, d_q, d_u, d_factors, d_ustar, (hipStream_t)stream);
}
