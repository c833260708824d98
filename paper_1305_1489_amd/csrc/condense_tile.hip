// Assembly + static condensation + scatter on the FP64 matrix cores (degrees 1..3).
//
// Same mathematics as k_condense (Sections 3-6; eq 3.55, 3.56, 4.5, 4.8, 4.10, 5.1-5.6,
// 6.5), organised as chains of 4x4x4 MFMA tile products with four elements per wavefront
// (one per matrix-core block).  The element dimension d3 is zero-padded to a multiple of
// 4 (padded diagonal entries of the SPD blocks set to 1); the trace dimension m = 4 d2 is
// always a multiple of 4 and is tiled without padding (a tile may straddle two faces, so
// face-dependent factors are applied per lane).
//   Gram      M  = P^T diag(|K| w / kappa) P,  Mc = P^T diag(|K| w c) P,  f = P^T (|K| w f)
//             (the quadrature index is the contraction dimension), + tauPP = sum_l T_l PP_l
//   Cholesky  M = U^T U (blocked, upper tiles in registers)
//   Z         = U^{-T} DP^T                   (block forward substitution, all faces)
//   for s in x, y, z:
//     W_s     = U^{-T} C_s^T,  C_s^T = sum_h a_{sh} Chat^{h T}
//     S      += W_s^T W_s
//     B      += n_{l s} W_s^T Z_l             (face l's columns)
//   B        += T_l DP_l^T
//   Cholesky  Mc + tauPP + sum W^T W = Us^T Us;   V = Us^{-T} [B | f]
//   C^K       = tauDD + (n_l . n_m) Z_l^T Z_m - V^T V,   Cf^K = V^T (Us^{-T} f)
// Each finished 4x4 tile of C^K is scattered straight into H (upper triangle mirrored,
// so H stays exactly symmetric); diagonal face blocks and F take atomic adds onto zeros.
// The factor store keeps U, Us (packed upper tiles) and f (tiles, column 0) per element.
#include <mutex>
#include <string>

#include "tile.h"

namespace hdg {
namespace {

template <int K>
struct TD {
  static constexpr int D3 = dim3(K), D2 = dim2(K), M = 4 * D2, NQD = (K + 2) * (K + 2) * (K + 2);
  static constexpr int T = (D3 + 3) / 4, MT = D2, QT = (NQD + 3) / 4;
  static constexpr int D3P4 = 4 * T, D2P4 = (D2 + 3) / 4 * 4, NQP = 4 * QT, NU = T * (T + 1) / 2;
  // factor store: U^{-1}, Us^{-1} (packed upper tiles), f, then the geometry record
  static constexpr int GEO_OFF = (2 * NU + T) * 16, FACTOR_LEN = GEO_OFF + G_REC;
};

// One geometry record per element, for the workspace form of the condensation: each
// thread computes its element's record into LDS, then the workgroup writes the (contiguous)
// records of its 64 elements with coalesced stores.
__global__ void __launch_bounds__(64) k_geo_records(hdg_mesh mesh, const double* __restrict__ tau,
                                                    double* __restrict__ rec, int du_removed) {
  __shared__ double s_rec[64 * G_REC];
  const int E0 = blockIdx.x * 64, E = E0 + threadIdx.x;
  if (E < mesh.nelt) tile_geo_record(E, mesh, tau, s_rec + threadIdx.x * G_REC, du_removed);
  __syncthreads();
  const int n = min(64, mesh.nelt - E0) * G_REC;
  double* out = rec + (size_t)E0 * G_REC;
  for (int i = threadIdx.x; i < n; i += 64) out[i] = s_rec[i];
}

// One group of four elements (w0 .. w0+3 of the work list) on one wavefront.  With DWS the
// diagonal face blocks and F entries of C^K, Cf^K go to the per-(element, face) buffer dws
// ([4 nelt][d2 (d2 + 1) / 2 + d2]: the row-packed upper triangle of the block, then the F
// entries) with plain stores, to be summed per face by k_diag_sum; without it
// they are atomic adds onto zeros.
using gdouble = __attribute__((address_space(1))) double;

//
// BDM selects the hybridized BDM element (Section 9, "BDM"): tau = 0 (the geometry records
// carry T_l = 0) and u in P_{k-1}(K).  Deleting the last d2 rows and columns of A1 (the
// degree-k modes of u and of its test space) is done by masking: those rows and columns of
// Mc and of C_s^T (so of W and S) and those entries of f are zero, with a unit diagonal in S,
// which decouples the removed modes (their rows of B and V vanish).
template <int K, bool DWS, bool BDM = false>
__device__ __forceinline__ void condense_tile_group(const hdg_mesh& mesh, const Tables& tb, const double* __restrict__ kappa,
                                                      const double* __restrict__ cco, const double* __restrict__ fco,
                                                      const double* __restrict__ tau, double* __restrict__ H,
                                                      double* __restrict__ F, double* __restrict__ factors,
                                                      const int* __restrict__ elems, int nwork,
                                                      double* __restrict__ Cout, double* __restrict__ Cfout, int w0, double* __restrict__ dws,
                                                      const double* __restrict__ geo_rec) {
  using D = TD<K>;
  constexpr int T = D::T, MT = D::MT, QT = D::QT, D3 = D::D3, D2 = D::D2, M = D::M;
  constexpr int NQD = D::NQD, NQP = D::NQP, NU = D::NU, D3P4 = D::D3P4, D2P4 = D::D2P4;
  __shared__ __attribute__((aligned(16))) double s_w[3][4][NQP + 1];  // +1: rows start in different banks
  __shared__ double s_geo[4][G_REC];
  __shared__ int s_slot[4][16];
  // workspace form: the 16 block base addresses (l, m) of each element of the group, the H
  // block of slot(l, m) for l != m and the element's own buffer block for l = m
  __shared__ double* s_base[DWS ? 4 : 1][16];
  __shared__ int s_fbe[4][4];
  __shared__ int s_E[4];
  __shared__ double s_x[64];
  __shared__ __attribute__((aligned(16))) double s_Z[T * MT][64];  // Z tiles, lane-contiguous
  {
    // lane-derived indices are recomputed per group and kept opaque to the compiler, so
    // that the many table addresses derived from them are not hoisted out of this loop
    // (hoisted, they outlive the register file and spill)
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    const int r = (lane >> 4) & 3, c = lane & 3, blk = (lane >> 2) & 3;
    __syncthreads();
    // the basis table of the Gram loop goes to the Z buffer (free until the Z phase) while
    // the geometry and coefficients load
    static_assert(lds_stage_bytes<NQP * D3P4>() <= (int)sizeof(s_Z), "Pt must fit in the Z buffer");
    double* s_pt = &s_Z[0][0];
    lds_stage<NQP * D3P4>(tb.Pt, s_pt, lane);
    constexpr int WIT = (4 * NQP + 63) / 64;
    double kv[WIT], cv[WIT], fv[WIT], vw[WIT];
    if constexpr (DWS) {
      // the precomputed geometry records, the block slots and the coefficients of the
      // group: every load is issued before any is used (the padding of a ragged last group
      // repeats its first element), so that all their latencies overlap in one round trip
      const auto elem = [&](int e) { return w0 + e < nwork ? w0 + e : w0; };
      static_assert(4 * G_REC % 64 == 0, "geometry records in whole passes");
      constexpr int GIT = 4 * G_REC / 64;
      double gv[GIT];
#pragma unroll
      for (int j = 0; j < GIT; ++j) {
        const int idx = lane + 64 * j;
        gv[j] = geo_rec[(size_t)elem(idx / G_REC) * G_REC + idx % G_REC];
      }
      const int sl = mesh.d_slot[16 * (size_t)elem(lane >> 4) + (lane & 15)];
#pragma unroll
      for (int it = 0; it < WIT; ++it) {
        const int idx = lane + 64 * it;
        const int e = min(idx / NQP, 3), q = idx % NQP;
        const bool ok = idx < 4 * NQP && q < NQD;
        const size_t o = ok ? (size_t)elem(e) * NQD + q : 0;
        kv[it] = kappa[o];
        cv[it] = cco[o];
        fv[it] = fco[o];
        vw[it] = tb.vol_w[ok ? q : 0];
      }
#pragma unroll
      for (int j = 0; j < GIT; ++j) (&s_geo[0][0])[lane + 64 * j] = gv[j];
      s_slot[lane >> 4][lane & 15] = sl;
      {
        const int l = (lane >> 2) & 3, m = lane & 3;
        s_base[lane >> 4][lane & 15] = l == m ? dws + (size_t)(4 * elem(lane >> 4) + l) * ws_block(D2)
                                              : H + (size_t)sl * D2 * D2;
      }
      if (lane < 4) s_E[lane] = elem(lane);
    } else {
      if (lane < 4) {
        const int wi = w0 + lane;
        int E = -1;
        if (wi < nwork) {
          E = elems ? elems[wi] : wi;
          if (E < 0 || E >= mesh.nelt) E = -1;
        }
        s_E[lane] = E;
        tile_geo_record(E, mesh, tau, s_geo[lane]);
      }
      {
        // face numbers and block slots: one (element, entry) per lane, loaded
        // unconditionally (clamped index) so that the loads of all lanes are in flight together
        const int e = lane >> 4, i = lane & 15;
        const int wi = w0 + e;
        int Ee = -1;
        if (wi < nwork) {
          Ee = elems ? elems[wi] : wi;
          if (Ee < 0 || Ee >= mesh.nelt) Ee = -1;
        }
        const size_t Es = Ee >= 0 ? (size_t)Ee : 0;
        const int sl = mesh.d_slot[16 * Es + i];
        const int fb = mesh.d_facebyele[4 * Es + (i & 3)];
        s_slot[e][i] = (Ee >= 0 && !Cout) ? sl : 0;
        if (i < 4) s_fbe[e][i] = Ee >= 0 ? fb : 0;
      }
      __syncthreads();
      // all the coefficient loads of the group are issued before any is used (indices
      // clamped instead of branched around), so that their latencies overlap
#pragma unroll
      for (int it = 0; it < WIT; ++it) {
        const int idx = lane + 64 * it;
        const int e = min(idx / NQP, 3), q = idx % NQP;
        const int Ee = s_E[e];
        const bool ok = idx < 4 * NQP && Ee >= 0 && q < NQD;
        const size_t o = ok ? (size_t)Ee * NQD + q : 0;
        kv[it] = kappa[o];
        cv[it] = cco[o];
        fv[it] = fco[o];
        vw[it] = tb.vol_w[ok ? q : 0];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < WIT; ++it) {
      const int idx = lane + 64 * it;
      const int e = min(idx / NQP, 3), q = idx % NQP;
      const bool ok = idx < 4 * NQP && s_E[e] >= 0 && q < NQD;
      const double wq = ok ? s_geo[e][G_VOL] * vw[it] : 0.0;
      if (idx < 4 * NQP) {
        s_w[0][e][q] = ok ? wq / kv[it] : 0.0;
        s_w[1][e][q] = wq * cv[it];
        s_w[2][e][q] = wq * fv[it];
      }
    }
    __syncthreads();
    const int E = s_E[blk];
    const double* geo = s_geo[blk];

    // ---- Gram matrices and the load vector (contraction over the quadrature points)
    double Ma[NU], Sa[NU], fa[T];
#pragma unroll
    for (int i = 0; i < NU; ++i) Ma[i] = Sa[i] = 0.0;
#pragma unroll
    for (int i = 0; i < T; ++i) fa[i] = 0.0;
    lds_stage_wait();
#pragma unroll 4
    for (int kq = 0; kq < QT; ++kq) {
      const int q = 4 * kq + r;
      double pv[T];
#pragma unroll
      for (int J = 0; J < T; ++J) pv[J] = s_pt[q * D3P4 + 4 * J + c];
      const double wk = s_w[0][blk][q], wc = s_w[1][blk][q], wf = s_w[2][blk][q];
#pragma unroll
      for (int N = 0; N < T; ++N) {
        const double yk = wk * pv[N], yc = wc * pv[N];
#pragma unroll
        for (int I = 0; I <= N; ++I) {
          Ma[utile(I, N, T)] = mfma4(pv[I], yk, Ma[utile(I, N, T)]);
          Sa[utile(I, N, T)] = mfma4(pv[I], yc, Sa[utile(I, N, T)]);
        }
      }
      const double yf = c == 0 ? wf : 0.0;
#pragma unroll
      for (int I = 0; I < T; ++I) fa[I] = mfma4(pv[I], yf, fa[I]);
    }
    // BDM: u lives in the first D3U modes
    constexpr int D3U = BDM ? D3 - D2 : D3;
    if constexpr (BDM) {
#pragma unroll
      for (int I = 0; I < T; ++I) fa[I] = 4 * I + r < D3U ? fa[I] : 0.0;
    }
    // the transposed Chat tables (element-independent) go to the weight buffer, dead from
    // here on, while the factorisations and the Z phase run
    constexpr int L3 = D3P4 * D3P4;
    static_assert(lds_stage_bytes<3 * L3>() <= (int)sizeof(s_w), "Chat tables must fit in the weight buffer");
    double* s_ct = &s_w[0][0][0];
    wave_lds_sync();
    lds_stage<3 * L3>(tb.ChatT, s_ct, lane);
    // tau PP (eq 4.5) and identity on the padded / unused part
    {
      // the table reads are all issued first (else the compiler recycles one register pair
      // and waits after each)
      constexpr int L4 = D3P4 * D3P4;
      double pp[NU][4];
#pragma unroll
      for (int I = 0; I < T; ++I)
#pragma unroll
        for (int N = I; N < T; ++N)
#pragma unroll
          for (int l = 0; l < 4; ++l) pp[utile(I, N, T)][l] = tb.PPt[l * L4 + (4 * I + r) * D3P4 + 4 * N + c];
      const double T0 = geo[G_T], T1 = geo[G_T + 1], T2 = geo[G_T + 2], T3 = geo[G_T + 3];
#pragma unroll
      for (int I = 0; I < T; ++I)
#pragma unroll
        for (int N = I; N < T; ++N) {
          const double* q = pp[utile(I, N, T)];
          const double sv = Sa[utile(I, N, T)] + (T0 * q[0] + T1 * q[1] + T2 * q[2] + T3 * q[3]);
          // selects, not branches (a branch here reshuffles the whole Gram state); the
          // workspace form has no empty slot (its padding repeats a real element)
          const bool empty = !DWS && E < 0;
          const bool unit = I == N && r == c && (4 * I + r >= D3 || empty);
          Ma[utile(I, N, T)] = unit ? 1.0 : (empty ? 0.0 : Ma[utile(I, N, T)]);
          // BDM: the removed u modes get a unit diagonal and no coupling
          const bool cut = BDM && (4 * I + r >= D3U || 4 * N + c >= D3U);
          const bool sunit = unit || (cut && I == N && r == c);
          Sa[utile(I, N, T)] = sunit ? 1.0 : ((empty || cut) ? 0.0 : sv);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    double Vd[T];
    tile_cholesky<T>(Ma, Vd, s_x);  // Ma <- U, M = U^T U
    double Ui[NU];
    tile_upper_inverse<T>(Ma, Vd, Ui);  // Ui = U^{-1}; L^{-1} = Ui^T
    __builtin_amdgcn_sched_barrier(0);

    // the trace-dimension column of lane c in tile N is j = 4N + c (face j / d2)
    // ---- Z = L^{-1} DP^T: Z(K,N) = sum_{J<=K} L^{-1}(K,J) DP^T(J,N)
#pragma unroll
    for (int N = 0; N < MT; ++N) {
      const int j = 4 * N + c, l = j / D2, i = j % D2;
      const double* dpt = tb.DPT + (size_t)((int)geo[G_MU + l] * 4 + l) * D3P4 * D2P4 + i;
      double rhs[T];
#pragma unroll
      for (int J = 0; J < T; ++J) rhs[J] = dpt[(4 * J + r) * D2P4];
#pragma unroll
      for (int Kk = 0; Kk < T; ++Kk) {
        double acc = 0.0;
#pragma unroll
        for (int J = 0; J <= Kk; ++J) acc = mfma4(Ui[utile(J, Kk, T)], rhs[J], acc);
        s_Z[Kk * MT + N][lane] = acc;
      }
    }
    __builtin_amdgcn_sched_barrier(0);

    // ---- W_s = L^{-1} C_s^T streamed by tile rows, the three directions together:
    // S += sum_s W_s^T W_s, and B += sum_s n_{ls} W_s^T Z_l = U_l^T Z_l with
    // U_l = sum_s n_{ls} W_s, so that each face's columns take one product per tile (two for
    // a tile whose columns straddle two faces, each with the other face's columns masked).
    lds_stage_wait();
    double B[T][MT];
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
      for (int N = 0; N < MT; ++N) B[I][N] = 0.0;
#pragma unroll
    for (int Kk = 0; Kk < T; ++Kk) {
      double Wr[3][T];
#pragma unroll
      for (int N = 0; N < T; ++N) {
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
#pragma unroll
        for (int J = 0; J <= Kk; ++J) {
          const int o = (4 * J + r) * D3P4 + 4 * N + c;
          const double h0 = s_ct[o], h1 = s_ct[L3 + o], h2 = s_ct[2 * L3 + o];
          const double u = Ui[utile(J, Kk, T)];
          double c0 = geo[G_A + 0] * h0 + geo[G_A + 1] * h1 + geo[G_A + 2] * h2;
          double c1 = geo[G_A + 3] * h0 + geo[G_A + 4] * h1 + geo[G_A + 5] * h2;
          double c2 = geo[G_A + 6] * h0 + geo[G_A + 7] * h1 + geo[G_A + 8] * h2;
          if constexpr (BDM) {  // columns of C_s^T beyond the u space of P_{k-1}
            const bool keep = 4 * N + c < D3U;
            c0 = keep ? c0 : 0.0;
            c1 = keep ? c1 : 0.0;
            c2 = keep ? c2 : 0.0;
          }
          acc0 = mfma4(u, c0, acc0);
          acc1 = mfma4(u, c1, acc1);
          acc2 = mfma4(u, c2, acc2);
        }
        Wr[0][N] = acc0;
        Wr[1][N] = acc1;
        Wr[2][N] = acc2;
      }
#pragma unroll
      for (int sd = 0; sd < 3; ++sd)
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
          for (int N = I; N < T; ++N) Sa[utile(I, N, T)] = mfma4(Wr[sd][I], Wr[sd][N], Sa[utile(I, N, T)]);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const double n0 = geo[G_N + 3 * l], n1 = geo[G_N + 3 * l + 1], n2 = geo[G_N + 3 * l + 2];
        double U[T];
#pragma unroll
        for (int I = 0; I < T; ++I) U[I] = n0 * Wr[0][I] + n1 * Wr[1][I] + n2 * Wr[2][I];
#pragma unroll
        for (int N = (l * D2) / 4; N <= ((l + 1) * D2 - 1) / 4; ++N) {
          const double z = s_Z[Kk * MT + N][lane];
          // columns 4N + c of this tile that belong to face l (all four, unless it straddles)
          const bool mine = (4 * N + c) / D2 == l;
          const bool whole = 4 * N >= l * D2 && 4 * N + 3 < (l + 1) * D2;
          const double zl = (whole || mine) ? z : 0.0;
#pragma unroll
          for (int I = 0; I < T; ++I) B[I][N] = mfma4(U[I], zl, B[I][N]);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    // B += T_l DP_l^T
#pragma unroll
    for (int N = 0; N < MT; ++N) {
      const int j = 4 * N + c, l = j / D2, i = j % D2;
      const double Tl = geo[G_T + l];
      const double* dpt = tb.DPT + (size_t)((int)geo[G_MU + l] * 4 + l) * D3P4 * D2P4 + i;
#pragma unroll
      for (int I = 0; I < T; ++I) B[I][N] += Tl * dpt[(4 * I + r) * D2P4];
    }
    __builtin_amdgcn_sched_barrier(0);

    // ---- factors kept for the reconstruction: U^{-1}, Us^{-1} (packed upper tiles), f
    double* fac = (factors && E >= 0) ? factors + (size_t)E * D::FACTOR_LEN : nullptr;
    const int ent = r * 4 + c;
    if (fac) {
#pragma unroll
      for (int i = 0; i < NU; ++i) fac[i * 16 + ent] = Ui[i];
#pragma unroll
      for (int i = 0; i < T; ++i) fac[(2 * NU + i) * 16 + ent] = fa[i];
      // the element's geometry record, for the reconstruction
      static_assert(G_REC % 16 == 0, "geometry record in whole 16-lane rows");
#pragma unroll
      for (int j = 0; j < G_REC / 16; ++j) fac[D::GEO_OFF + 16 * j + ent] = geo[16 * j + ent];
    }

    // ---- Cholesky of S, Us^{-1}, and V = Ls^{-1} [B | f] (rows from the bottom, in place)
    double Vs[T];
    tile_cholesky<T>(Sa, Vs, s_x);
    tile_upper_inverse<T>(Sa, Vs, Ui);  // Ui now holds Us^{-1}
    if (fac) {
#pragma unroll
      for (int i = 0; i < NU; ++i) fac[(NU + i) * 16 + ent] = Ui[i];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int Kk = T - 1; Kk >= 0; --Kk) {
#pragma unroll
      for (int N = 0; N < MT; ++N) {
        double acc = 0.0;
#pragma unroll
        for (int J = 0; J <= Kk; ++J) acc = mfma4(Ui[utile(J, Kk, T)], B[J][N], acc);
        B[Kk][N] = acc;
      }
      double acc = 0.0;
#pragma unroll
      for (int J = 0; J <= Kk; ++J) acc = mfma4(Ui[utile(J, Kk, T)], fa[J], acc);
      fa[Kk] = acc;
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (DWS) {
      // ---- C^K tiles and Cf^K into H (off-diagonal face blocks) and the per-(element, face)
      // buffer (diagonal blocks, F).  Each tile row first runs all of its products, then
      // stores whose block addresses come from the table built at set-up: no branch splits
      // a row, so the products of one row overlap the stores of the previous one.
      double* const* base = s_base[blk];
#pragma unroll
      for (int I = 0; I < MT; ++I) {
        const int a = 4 * I + r, la = a / D2, ia = a % D2;
        const double tl = geo[G_T + la];
        double zi[T];
#pragma unroll
        for (int Kk = 0; Kk < T; ++Kk) zi[Kk] = s_Z[Kk * MT + I][lane];
        double val[MT];
#pragma unroll
        for (int N = I; N < MT; ++N) {
          double g1 = 0.0, g2 = 0.0;
#pragma unroll
          for (int Kk = 0; Kk < T; ++Kk) {
            g1 = mfma4(zi[Kk], s_Z[Kk * MT + N][lane], g1);
            g2 = mfma4(B[Kk][I], B[Kk][N], g2);
          }
          const int b = 4 * N + c, lb = b / D2;
          val[N] = geo[G_NN + 4 * la + lb] * g1 - g2 + (a == b ? tl : 0.0);
        }
        double h = 0.0;
#pragma unroll
        for (int Kk = 0; Kk < T; ++Kk) h = mfma4(B[Kk][I], fa[Kk], h);
#pragma unroll
        for (int N = I; N < MT; ++N) {
          const int b = 4 * N + c, lb = b / D2, ib = b % D2;
          // lane (r, c) now holds the upper entry (a2, b2) = (4I + c, 4N + r), stored mirrored
          const double tv = tile_transpose(val[N]);
          const int a2 = 4 * I + c, b2 = 4 * N + r, la2 = a2 / D2, lb2 = b2 / D2;
          const int ia2 = a2 % D2, ib2 = b2 % D2;
          // off-diagonal blocks: row-major in H; the element's diagonal blocks: row-packed
          // upper triangle in the workspace (the mirror of an upper entry lands on that
          // same entry, written twice with one value)
          const int o1 = la == lb ? ia * D2 - ia * (ia - 1) / 2 + (ib - ia) : ia * D2 + ib;
          const int o2 = la2 == lb2 ? ia2 * D2 - ia2 * (ia2 - 1) / 2 + (ib2 - ia2) : ib2 * D2 + ia2;
          // the table holds generic pointers; stored through as global ones, so these are
          // global stores (a flat store also counts against the LDS wait counter, and every
          // later LDS wait of the loop would then wait for the store to reach memory)
          gdouble* p1 = (gdouble*)(base[4 * la + lb]) + o1;
          gdouble* p2 = (gdouble*)(base[4 * lb2 + la2]) + o2;
          if (I != N || r <= c) *p1 = val[N];
          if (I != N || c < r) *p2 = tv;
        }
        if (c == 0) ((gdouble*)(base[5 * la]))[D2 * (D2 + 1) / 2 + ia] = h;
      }
    } else {
      // ---- C^K tiles and Cf^K, straight to H and F (or to the export arrays)
#pragma unroll
      for (int I = 0; I < MT; ++I) {
        const int a = 4 * I + r, la = a / D2, ia = a % D2;
        double zi[T];
#pragma unroll
        for (int Kk = 0; Kk < T; ++Kk) zi[Kk] = s_Z[Kk * MT + I][lane];
#pragma unroll
        for (int N = I; N < MT; ++N) {
          double g1 = 0.0, g2 = 0.0;
#pragma unroll
          for (int Kk = 0; Kk < T; ++Kk) {
            g1 = mfma4(zi[Kk], s_Z[Kk * MT + N][lane], g1);
            g2 = mfma4(B[Kk][I], B[Kk][N], g2);
          }
          const int b = 4 * N + c, lb = b / D2, ib = b % D2;
          double val = geo[G_NN + 4 * la + lb] * g1 - g2;
          if (a == b) val += geo[G_T + la];
          // only entries of the upper triangle (a <= b) are ever written; their mirror images
          // are written from the transposed tile, so each 4-lane row of a store is contiguous
          const double tv = tile_transpose(val);  // lane (r, c) now holds C[4I + c][4N + r]
          if (E >= 0 && (I != N || r <= c)) {
            if (Cout) {
              const size_t base = (size_t)(w0 + blk) * M * M;
              Cout[base + (size_t)a * M + b] = val;
              Cout[base + (size_t)b * M + a] = val;
            } else {
              const size_t s1 = s_slot[blk][4 * la + lb];
              if (la == lb) {
                unsafeAtomicAdd(&H[(s1 * D2 + ia) * D2 + ib], val);
                if (ia != ib) unsafeAtomicAdd(&H[(s1 * D2 + ib) * D2 + ia], val);
              } else {
                H[(s1 * D2 + ia) * D2 + ib] = val;
              }
            }
          }
          {
            const int a2 = 4 * I + c, b2 = 4 * N + r;  // the upper entry now held by this lane
            const int la2 = a2 / D2, lb2 = b2 / D2;
            if (!Cout && E >= 0 && (I != N || c <= r) && la2 != lb2) {
              const size_t s2 = s_slot[blk][4 * lb2 + la2];
              H[(s2 * D2 + b2 % D2) * D2 + a2 % D2] = tv;
            }
          }
        }
        double h = 0.0;
#pragma unroll
        for (int Kk = 0; Kk < T; ++Kk) h = mfma4(B[Kk][I], fa[Kk], h);
        if (E >= 0 && c == 0) {
          if (Cfout)
            Cfout[(size_t)(w0 + blk) * M + a] = h;
          else
            unsafeAtomicAdd(&F[(size_t)s_fbe[blk][la] * D2 + ia], h);
        }
      }
    }
  }
}

// EXPORT selects the debugging form (listed elements, C^K and Cf^K written out instead of
// scattered); the scatter form is compiled with those pointers known to be null.
template <int K, bool EXPORT, bool DWS, bool BDM = false>
__global__ void __launch_bounds__(64) k_condense_tile(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                      const double* __restrict__ cco, const double* __restrict__ fco,
                                                      const double* __restrict__ tau, double* __restrict__ H,
                                                      double* __restrict__ F, double* __restrict__ factors,
                                                      const int* __restrict__ elems, int nwork,
                                                      double* __restrict__ Cout, double* __restrict__ Cfout,
                                                      int xcd_remap, double* __restrict__ dws,
                                                      const double* __restrict__ geo_rec) {
  for (int w0 = batch_block(xcd_remap) * 4; w0 < nwork; w0 += gridDim.x * 4)
    condense_tile_group<K, DWS, BDM>(mesh, tb, kappa, cco, fco, tau, H, F, factors, EXPORT ? elems : nullptr, nwork,
                                EXPORT ? Cout : nullptr, EXPORT ? Cfout : nullptr, w0, dws, DWS ? geo_rec : nullptr);
}

// Persistent batched form: work unit u is group u - unit_begin of its mesh.
template <int K>
__global__ void __launch_bounds__(64) k_batch_condense_tile(const BatchItem* __restrict__ items, int nitems,
                                                            int total_units, Tables tb, int xcd_remap) {
  for (int u = batch_block(xcd_remap); u < total_units; u += gridDim.x) {
    const BatchItem* it = items + batch_find(items, nitems, u);
    condense_tile_group<K, false>(as_global(it->mesh), tb, as_global(it->kappa), as_global(it->c), as_global(it->f),
                                  as_global(it->tau), as_global(it->H), as_global(it->F), as_global(it->factors),
                                  nullptr, (int)it->mesh.nelt, nullptr, nullptr, 4 * (u - it->unit_begin), nullptr,
                                  nullptr);
  }
}

template <int D2>
__global__ void k_zero_diag_t(const int* __restrict__ diag, int nfc, double* __restrict__ H, double* __restrict__ F) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)nfc * D2 * D2) return;
  const size_t f = i / (D2 * D2), e = i % (D2 * D2);
  H[(size_t)diag[f] * D2 * D2 + e] = 0.0;
  if (e < D2) F[f * D2 + e] = 0.0;
}

// H_ff (diagonal block) and F_f from the per-(element, face) contributions of the (one or
// two) elements holding face f, in a fixed order; (0 + a) + b equals the atomic result.
// One packed entry per thread (contiguous reads of both contributions); an off-diagonal
// entry of the block is written to both of its mirrored places.
template <int D2>
__global__ void k_diag_sum(const int* __restrict__ diag, const int* __restrict__ face_elem, int nfc,
                           const double* __restrict__ dws, double* __restrict__ H, double* __restrict__ F) {
  constexpr int W = ws_block(D2), TRI = D2 * (D2 + 1) / 2;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)nfc * W) return;
  const int f = (int)(i / W);
  const int p = (int)(i - (int64_t)f * W);
  const int v0 = face_elem[2 * f], v1 = face_elem[2 * f + 1];
  double v = 0.0 + dws[(size_t)v0 * W + p];
  if (v1 >= 0) v += dws[(size_t)v1 * W + p];
  if (p < TRI) {
    // packed (x, y), x <= y: rows x hold D2 - x entries
    int x = 0, rem = p;
#pragma unroll
    for (int r = 0; r < D2 - 1; ++r)
      if (rem >= D2 - x) {
        rem -= D2 - x;
        ++x;
      }
    const int y = x + rem;
    double* blk = H + (size_t)diag[f] * D2 * D2;
    blk[x * D2 + y] = v;
    if (y != x) blk[y * D2 + x] = v;
  } else {
    F[(size_t)f * D2 + (p - TRI)] = v;
  }
}

template <int K>
hdg_status run_condense_tile(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                             const double* f, const double* tau, double* H, double* F, double* factors,
                             const int* elems, int64_t n, double* Cout, double* Cfout, double* dws, hipStream_t s) {
  using D = TD<K>;
  if (!Cout && !dws) {
    const size_t tot = (size_t)mesh->nfc * D::D2 * D::D2;
    k_zero_diag_t<D::D2><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(mesh->d_diag, (int)mesh->nfc, H, F);
    HDG_CHECK_LAUNCH("k_zero_diag");
  }
  if (n == 0) return HDG_OK;
  const int64_t groups = (n + 3) / 4;
  const hdg_tile_config lc = launch_config(K);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(groups, (int64_t)lc.workgroups_per_cu * device_cu_count()));
  if (Cout) {
    k_condense_tile<K, true, false><<<grid, 64, 0, s>>>(*mesh, disc->dev, kappa, c, f, tau, H, F, factors, elems,
                                                        (int)n, Cout, Cfout, lc.xcd_remap, nullptr, nullptr);
  } else if (dws) {
    double* geo_rec = reinterpret_cast<double*>(reinterpret_cast<char*>(dws) + condense_ws_geo_offset(D::D2, mesh->nelt));
    timer_begin("k_geo_records", s);
    k_geo_records<<<(unsigned)((mesh->nelt + 63) / 64), 64, 0, s>>>(*mesh, tau, geo_rec, 0);
    timer_end("k_geo_records", s);
    timer_begin("k_condense_tile", s);
    k_condense_tile<K, false, true><<<grid, 64, 0, s>>>(*mesh, disc->dev, kappa, c, f, tau, H, F, factors, elems,
                                                        (int)n, Cout, Cfout, lc.xcd_remap, dws, geo_rec);
    timer_end("k_condense_tile", s);
    const size_t tot = (size_t)mesh->nfc * ws_block(D::D2);
    timer_begin("k_diag_sum", s);
    k_diag_sum<D::D2><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(mesh->d_diag, mesh->d_face_elem, (int)mesh->nfc,
                                                                     dws, H, F);
    timer_end("k_diag_sum", s);
  } else {
    timer_begin("k_condense_tile", s);
    k_condense_tile<K, false, false><<<grid, 64, 0, s>>>(*mesh, disc->dev, kappa, c, f, tau, H, F, factors, elems,
                                                         (int)n, Cout, Cfout, lc.xcd_remap, nullptr, nullptr);
    timer_end("k_condense_tile", s);
  }
  HDG_CHECK_LAUNCH("k_condense_tile");
  return HDG_OK;
}

// ---- the library's own workspace for callers that cannot allocate (hdg_assemble_condense_noalloc)
//
// A file-scope device array: the runtime gives every device the library runs on its own
// copy when the code object is loaded, and it lives until the process ends.  In host code
// `scratch` names a host-side stand-in, not a device address: the device address is
// looked up per device with hipGetSymbolAddress and only that pointer is ever handed to a
// kernel.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on the first call on each device).
hdg_status scratch_pointer(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return check_hip(e, "hdg_assemble_condense_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(HDG_ERR_DEVICE, "hdg_assemble_condense_noalloc: device index beyond the supported range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return check_hip(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                "hdg_assemble_condense_noalloc: hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return HDG_OK;
}

// The hybridized BDM element (workspace form only): records with T_l = 0 and d2 removed u
// modes, the masked group kernel, the per-face sums.
template <int K>
hdg_status run_condense_tile_bdm(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                                 const double* f, double* H, double* F, double* factors, double* dws, hipStream_t s) {
  using D = TD<K>;
  const int64_t n = mesh->nelt, groups = (n + 3) / 4;
  const hdg_tile_config lc = launch_config(K);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(groups, (int64_t)lc.workgroups_per_cu * device_cu_count()));
  double* geo_rec = reinterpret_cast<double*>(reinterpret_cast<char*>(dws) + condense_ws_geo_offset(D::D2, mesh->nelt));
  k_geo_records<<<(unsigned)((mesh->nelt + 63) / 64), 64, 0, s>>>(*mesh, nullptr, geo_rec, D::D2);
  timer_begin("k_condense_tile", s);
  k_condense_tile<K, false, true, true><<<grid, 64, 0, s>>>(*mesh, disc->dev, kappa, c, f, nullptr, H, F, factors,
                                                            nullptr, (int)n, nullptr, nullptr, lc.xcd_remap, dws,
                                                            geo_rec);
  timer_end("k_condense_tile", s);
  const size_t tot = (size_t)mesh->nfc * ws_block(D::D2);
  k_diag_sum<D::D2><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(mesh->d_diag, mesh->d_face_elem, (int)mesh->nfc,
                                                                   dws, H, F);
  HDG_CHECK_LAUNCH("k_condense_tile (BDM)");
  return HDG_OK;
}

}  // namespace

hdg_status dispatch_condense_tile_bdm(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                                      const double* f, double* H, double* F, double* factors, double* dws,
                                      hipStream_t s) {
  switch (disc->host.k) {
    case 1: return run_condense_tile_bdm<1>(disc, mesh, kappa, c, f, H, F, factors, dws, s);
    case 2: return run_condense_tile_bdm<2>(disc, mesh, kappa, c, f, H, F, factors, dws, s);
    case 3: return run_condense_tile_bdm<3>(disc, mesh, kappa, c, f, H, F, factors, dws, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_assemble_condense_bdm: degrees 1..3");
}

size_t condense_scratch_capacity() { return kScratchBytes; }

hdg_status condense_static_workspace(size_t need, double** ws) {
  *ws = nullptr;
  if (need > kScratchBytes)
    return set_error(HDG_ERR_WORKSPACE, "hdg_assemble_condense_noalloc: the mesh needs " + std::to_string(need) +
                                            " bytes of workspace, more than the library's static " +
                                            std::to_string(kScratchBytes) + " bytes");
  if (need == 0) return HDG_OK;
  return scratch_pointer(ws);
}

int tile_factor_len(int k) {
  switch (k) {
    case 1: return TD<1>::FACTOR_LEN;
    case 2: return TD<2>::FACTOR_LEN;
    case 3: return TD<3>::FACTOR_LEN;
  }
  return 0;
}

hdg_status launch_batch_condense_tile(int k, const Tables& tb, const BatchItem* d_items, int nitems, int total_units,
                                      int grid, int xcd_remap, hipStream_t s) {
  switch (k) {
    case 1: k_batch_condense_tile<1><<<grid, 64, 0, s>>>(d_items, nitems, total_units, tb, xcd_remap); break;
    case 2: k_batch_condense_tile<2><<<grid, 64, 0, s>>>(d_items, nitems, total_units, tb, xcd_remap); break;
    case 3: k_batch_condense_tile<3><<<grid, 64, 0, s>>>(d_items, nitems, total_units, tb, xcd_remap); break;
    default: return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "batched tile condensation: unsupported degree");
  }
  HDG_CHECK_LAUNCH("k_batch_condense_tile");
  return HDG_OK;
}

hdg_status dispatch_condense_tile(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                                  const double* f, const double* tau, double* H, double* F, double* factors,
                                  const int* elems, int64_t n, double* Cout, double* Cfout, double* dws,
                                  hipStream_t s) {
  switch (disc->host.k) {
    case 1: return run_condense_tile<1>(disc, mesh, kappa, c, f, tau, H, F, factors, elems, n, Cout, Cfout, dws, s);
    case 2: return run_condense_tile<2>(disc, mesh, kappa, c, f, tau, H, F, factors, elems, n, Cout, Cfout, dws, s);
    case 3: return run_condense_tile<3>(disc, mesh, kappa, c, f, tau, H, F, factors, elems, n, Cout, Cfout, dws, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "tile condensation: unsupported degree");
}

}  // namespace hdg
