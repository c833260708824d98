// Assembly of the element blocks, static condensation onto the four face traces, and
// scatter into the global trace system (Sections 3-6 of the paper).
//
// Per element K (one wavefront, blocks resident in LDS):
//   volume terms (eq 3.55, eq 3.56):
//     M  = sum_q |K| w_q kappa_q^{-1} p_q p_q^T,   Mc = sum_q |K| w_q c_q p_q p_q^T,
//     f  = sum_q |K| w_q f_q p_q,                  C_s = sum_h a_{s h} Chat^h
//   face terms (eq 4.5, 4.10, 4.8): tauPP = sum_l T_l PP_l, DP_l = DP_{perm(K,l), l},
//     tauDP_l = T_l DP_l, n_sDP_l = n_{l s} DP_l, tauDD = diag(T_l I)
//   condensation of eq 5.5-5.6 by block elimination of q, exploiting that A1 is
//   symmetric up to the sign of its last block row:
//     L L^T = M;  W_s = L^{-1} C_s^T;  S = Mc + tauPP + sum_s W_s^T W_s = Ls Ls^T;
//     Z_l = L^{-1} DP_l^T;  B_l = T_l DP_l^T + (sum_s n_{l s} W_s)^T Z_l;  V = Ls^{-1} B;
//     C^K = tauDD + [ (n_l . n_m) Z_l^T Z_m ]_{lm} - V^T V,   Cf^K = V^T Ls^{-1} f.
//   Only the upper triangle of C^K is formed; it is mirrored, so H is exactly symmetric.
// Scatter (eq 6.5): the (l, m) block of C^K goes to block slot[K][4l+m] of H; off-diagonal
// blocks have a single writer, diagonal blocks and F at most two (atomic adds onto zeros,
// which are order-independent for two addends).
#include "device_common.h"

namespace hdg {
namespace {

// Right-looking Cholesky in place on the lower triangle of the row-major N x N matrix A
// (leading dimension ld), by the whole workgroup: pass j applies column j (still unscaled,
// L_ij L_kj = A_ij A_kj / A_jj) to the trailing triangle and scales column j - 1, whose
// last reader was the pass before, so each column costs one barrier.
template <int N>
__device__ inline void wg_cholesky(double* A, int ld) {
  const int t = threadIdx.x, nt = blockDim.x;
  double prev = 1.0;  // pivot of column j - 1, read before anyone rescaled it
  for (int j = 0; j < N; ++j) {
    const double piv = A[j * ld + j];
    const double ip = 1.0 / piv;
    const int m = N - 1 - j;
    for (int p = t; p < m * m; p += nt) {
      const int i = j + 1 + p / m, k = j + 1 + p % m;
      if (k <= i) A[i * ld + k] -= A[i * ld + j] * A[k * ld + j] * ip;
    }
    if (j > 0) {
      const double d = sqrt(prev), id = 1.0 / d;
      for (int i = j - 1 + t; i < N; i += nt) A[i * ld + j - 1] = i == j - 1 ? d : A[i * ld + j - 1] * id;
    }
    prev = piv;
    __syncthreads();
  }
  const double d = sqrt(prev);
  if (t == 0) A[(N - 1) * ld + N - 1] = d;
  __syncthreads();
}

// X <- L^{-1} X for the columns of one or two row-major blocks of N rows (block b: nc[b]
// columns; row r, column c at X[b] + (c / cs[b]) * ss[b] + r * ld[b] + c % cs[b], which
// lets three stacked N x N blocks act as one), right-looking: pass k eliminates row k
// (unscaled) from the rows below and scales row k - 1.  L lower triangular, factor diagonal.
template <int N>
__device__ inline void wg_forward(const double* L, int ldl, double* X0, int ld0, int nc0, int cs0, int ss0,
                                  double* X1, int ld1, int nc1) {
  const int t = threadIdx.x, nt = blockDim.x, nc = nc0 + nc1;
  auto at = [&](int r, int c) -> double& {
    return c < nc0 ? X0[(c / cs0) * ss0 + r * ld0 + c % cs0] : X1[r * ld1 + (c - nc0)];
  };
  double iprev = 1.0;
  for (int k = 0; k < N; ++k) {
    const double ik = 1.0 / L[k * ldl + k];
    const int m = N - 1 - k;
    for (int p = t; p < m * nc; p += nt) {
      const int r = k + 1 + p / nc, c = p % nc;
      at(r, c) -= L[r * ldl + k] * at(k, c) * ik;
    }
    if (k > 0)
      for (int c = t; c < nc; c += nt) at(k - 1, c) *= iprev;
    iprev = ik;
    __syncthreads();
  }
  for (int c = t; c < nc; c += nt) at(N - 1, c) *= iprev;
  __syncthreads();
}

template <int K>
struct CondenseSmem {
  using Dm = Dims<K>;
  double wk[Dm::NQD], wc[Dm::NQD], wf[Dm::NQD];
  double L[Dm::D3 * Dm::D3];
  double S[Dm::D3 * Dm::D3];
  double W[3 * Dm::D3 * Dm::D3];
  double Z[Dm::D3 * Dm::M];
  double V[Dm::D3 * (Dm::M + 1)];  // B (then V) with the f column appended
  double U[Dm::D3 * Dm::D3];
};

// Work item w (one element) on one wavefront.
template <int K>
__device__ __forceinline__ void condense_element(const hdg_mesh& mesh, const Tables& tb, const double* __restrict__ kappa,
                                                 const double* __restrict__ cco, const double* __restrict__ fco,
                                                 const double* __restrict__ tau, double* __restrict__ H,
                                                 double* __restrict__ F, double* __restrict__ factors,
                                                 const int* __restrict__ elems, int nwork, double* __restrict__ Cout,
                                                 double* __restrict__ Cfout, int w) {
  using Dm = Dims<K>;
  constexpr int D3 = Dm::D3, D2 = Dm::D2, M = Dm::M, NQD = Dm::NQD, MV = M + 1;
  __shared__ CondenseSmem<K> sm;
  const int t = threadIdx.x, nt = blockDim.x;
  {
    const int E = elems ? elems[w] : w;
    if (E < 0 || E >= mesh.nelt) return;  // uniform across the block
    ElemGeom g;
    load_geometry(E, mesh, tau, g);
    // ---- coefficients at the quadrature points
    for (int q = t; q < NQD; q += nt) {
      double wq = g.vol * tb.vol_w[q];
      sm.wk[q] = wq / kappa[(size_t)E * NQD + q];
      sm.wc[q] = wq * cco[(size_t)E * NQD + q];
      sm.wf[q] = wq * fco[(size_t)E * NQD + q];
    }
    __syncthreads();
    // ---- Gram matrices (upper triangle, mirrored) and the load vector.  The basis table
    // is staged in LDS in chunks of points (in the Z / V / U space, free until the
    // solves); one thread per upper pair (i, j), pairs numbered from the last row up.
    {
      constexpr int QC = (NQD + 1) / 2, NP = D3 * (D3 + 1) / 2;
      static_assert(QC * D3 <= D3 * M + D3 * (M + 1) + D3 * D3, "basis chunk must fit the solve buffers");
      double* sP = sm.Z;  // Z, V and U are consecutive
      for (int q0 = 0; q0 < NQD; q0 += QC) {
        const int nq = min(QC, NQD - q0);
        for (int i = t; i < nq * D3; i += nt) sP[i] = tb.P[q0 * D3 + i];
        __syncthreads();
        for (int pp = t; pp < NP; pp += nt) {
          const int kk = NP - 1 - pp;
          int rr = (int)((sqrtf(8.0f * kk + 1.0f) - 1.0f) * 0.5f);
          while (rr * (rr + 1) / 2 > kk) --rr;
          while ((rr + 1) * (rr + 2) / 2 <= kk) ++rr;
          const int i = D3 - 1 - rr, j = D3 - 1 - (kk - rr * (rr + 1) / 2);
          double sk = 0, sc = 0;
#pragma unroll 4
          for (int q = 0; q < nq; ++q) {
            const double pq = sP[q * D3 + i] * sP[q * D3 + j];
            sk += sm.wk[q0 + q] * pq;
            sc += sm.wc[q0 + q] * pq;
          }
          if (q0 == 0) {
            for (int l = 0; l < 4; ++l) sc += g.T[l] * tb.PP[(l * D3 + i) * D3 + j];
          } else {
            sk += sm.L[i * D3 + j];
            sc += sm.S[i * D3 + j];
          }
          sm.L[i * D3 + j] = sk;
          sm.L[j * D3 + i] = sk;
          sm.S[i * D3 + j] = sc;
          sm.S[j * D3 + i] = sc;
        }
        __syncthreads();
      }
    }
    for (int i = t; i < D3; i += nt) {
      double s = 0;
      for (int q = 0; q < NQD; ++q) s += sm.wf[q] * tb.P[q * D3 + i];
      sm.V[i * MV + M] = s;  // f in the last column of V
    }
    // ---- W_s = C_s^T (before the solve): W[s][r][i] = sum_h a[s][h] Chat[h][i][r]
    for (int idx = t; idx < 3 * D3 * D3; idx += nt) {
      const int s = idx / (D3 * D3), r = (idx / D3) % D3, i = idx % D3;
      double v = 0;
      for (int h = 0; h < 3; ++h) v += g.a[s][h] * tb.Chat[(h * D3 + i) * D3 + r];
      sm.W[idx] = v;
    }
    // ---- Z_l = DP_l^T (before the solve)
    for (int idx = t; idx < D3 * M; idx += nt) {
      const int r = idx / M, c = idx % M, l = c / D2, i = c % D2;
      sm.Z[idx] = tb.DP[((g.mu[l] * 4 + l) * D2 + i) * D3 + r];
    }
    __syncthreads();
    wg_cholesky<D3>(sm.L, D3);
    // W = L^{-1} C^T (three stacked D3 x D3 blocks) and Z = L^{-1} DP^T, in one sweep
    wg_forward<D3>(sm.L, D3, sm.W, D3, 3 * D3, D3, D3 * D3, sm.Z, M, M);
    // ---- S += sum_s W_s^T W_s
    for (int idx = t; idx < D3 * D3; idx += nt) {
      const int i = idx / D3, j = idx % D3;
      if (j < i) continue;
      double s = 0;
      for (int c = 0; c < 3; ++c)
        for (int r = 0; r < D3; ++r) s += sm.W[(c * D3 + r) * D3 + i] * sm.W[(c * D3 + r) * D3 + j];
      sm.S[i * D3 + j] += s;
      if (j != i) sm.S[j * D3 + i] += s;
    }
    __syncthreads();
    wg_cholesky<D3>(sm.S, D3);
    // ---- B_l = T_l DP_l^T + U_l^T Z_l with U_l = sum_s n_{l s} W_s
    for (int l = 0; l < 4; ++l) {
      for (int idx = t; idx < D3 * D3; idx += nt)
        sm.U[idx] = g.n[l][0] * sm.W[idx] + g.n[l][1] * sm.W[D3 * D3 + idx] + g.n[l][2] * sm.W[2 * D3 * D3 + idx];
      __syncthreads();
      for (int idx = t; idx < D3 * D2; idx += nt) {
        const int i = idx / D2, c = l * D2 + idx % D2;
        double s = g.T[l] * tb.DP[((g.mu[l] * 4 + l) * D2 + (idx % D2)) * D3 + i];
        for (int r = 0; r < D3; ++r) s += sm.U[r * D3 + i] * sm.Z[r * M + c];
        sm.V[i * MV + c] = s;
      }
      __syncthreads();
    }
    // ---- V = Ls^{-1} [B | f]
    wg_forward<D3>(sm.S, D3, sm.V, MV, MV, MV, 0, nullptr, 0, 0);
    // ---- C^K (upper triangle) and Cf^K; scatter or export
    for (int idx = t; idx < M * M; idx += nt) {
      const int a = idx / M, b = idx % M;
      if (b < a) continue;
      const int la = a / D2, lb = b / D2, ia = a % D2, ib = b % D2;
      double zz = 0, vv = 0;
      for (int r = 0; r < D3; ++r) {
        zz += sm.Z[r * M + a] * sm.Z[r * M + b];
        vv += sm.V[r * MV + a] * sm.V[r * MV + b];
      }
      const double nn = g.n[la][0] * g.n[lb][0] + g.n[la][1] * g.n[lb][1] + g.n[la][2] * g.n[lb][2];
      double c = nn * zz - vv;
      if (a == b) c += g.T[la];
      if (Cout) {
        Cout[((size_t)w * M + a) * M + b] = c;
        Cout[((size_t)w * M + b) * M + a] = c;
      } else {
        const size_t s1 = mesh.d_slot[16 * E + 4 * la + lb];
        if (la == lb) {
          unsafeAtomicAdd(&H[(s1 * D2 + ia) * D2 + ib], c);
          if (ia != ib) unsafeAtomicAdd(&H[(s1 * D2 + ib) * D2 + ia], c);
        } else {
          const size_t s2 = mesh.d_slot[16 * E + 4 * lb + la];
          H[(s1 * D2 + ia) * D2 + ib] = c;
          H[(s2 * D2 + ib) * D2 + ia] = c;
        }
      }
    }
    for (int a = t; a < M; a += nt) {
      double s = 0;
      for (int r = 0; r < D3; ++r) s += sm.V[r * MV + a] * sm.V[r * MV + M];
      if (Cfout) {
        Cfout[(size_t)w * M + a] = s;
      } else {
        const int la = a / D2, ia = a % D2;
        unsafeAtomicAdd(&F[(size_t)mesh.d_facebyele[4 * E + la] * D2 + ia], s);
      }
    }
    // ---- factors kept for the reconstruction: packed L, packed Ls, f
    if (factors) {
      double* fa = factors + (size_t)E * (D3 * (D3 + 1) + D3);
      for (int idx = t; idx < D3 * D3; idx += nt) {
        const int i = idx / D3, j = idx % D3;
        if (j > i) continue;
        fa[i * (i + 1) / 2 + j] = sm.L[idx];
        fa[D3 * (D3 + 1) / 2 + i * (i + 1) / 2 + j] = sm.S[idx];
      }
      // f itself (the solve above overwrote it by Ls^{-1} f): recompute it
      for (int i = t; i < D3; i += nt) {
        double s = 0;
        for (int q = 0; q < NQD; ++q) s += sm.wf[q] * tb.P[q * D3 + i];
        fa[D3 * (D3 + 1) + i] = s;
      }
    }
    __syncthreads();
  }
}

// EXPORT selects the debugging form (listed elements, C^K and Cf^K written out instead of
// scattered); the scatter form is compiled with those pointers known to be null.
template <int K, int NT, bool EXPORT>
__global__ void __launch_bounds__(NT) k_condense(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                 const double* __restrict__ cco, const double* __restrict__ fco,
                                                 const double* __restrict__ tau, double* __restrict__ H,
                                                 double* __restrict__ F, double* __restrict__ factors,
                                                 const int* __restrict__ elems, int nwork, double* __restrict__ Cout,
                                                 double* __restrict__ Cfout, int xcd_remap) {
  for (int w = batch_block(xcd_remap); w < nwork; w += gridDim.x)
    condense_element<K>(mesh, tb, kappa, cco, fco, tau, H, F, factors, EXPORT ? elems : nullptr, nwork,
                        EXPORT ? Cout : nullptr, EXPORT ? Cfout : nullptr, w);
}

// Persistent batched form: work unit u is element u - unit_begin of its mesh.
template <int K, int NT>
__global__ void __launch_bounds__(NT) k_batch_condense(const BatchItem* __restrict__ items, int nitems, int total_units,
                                                       Tables tb, int xcd_remap) {
  for (int u = batch_block(xcd_remap); u < total_units; u += gridDim.x) {
    const BatchItem* it = items + batch_find(items, nitems, u);
    condense_element<K>(it->mesh, tb, it->kappa, it->c, it->f, it->tau, it->H, it->F, it->factors, nullptr,
                        (int)it->mesh.nelt, nullptr, nullptr, u - it->unit_begin);
  }
}

// Zero the diagonal blocks of H and F before the scatter.
template <int D2>
__global__ void k_zero_diag(const int* __restrict__ diag, int nfc, double* __restrict__ H, double* __restrict__ F) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)nfc * D2 * D2) return;
  const size_t f = i / (D2 * D2), e = i % (D2 * D2);
  H[(size_t)diag[f] * D2 * D2 + e] = 0.0;
  if (e < D2) F[f * D2 + e] = 0.0;
}

template <int K>
hdg_status run_condense(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                        const double* f, const double* tau, double* H, double* F, double* factors,
                        const int* elems, int64_t n, double* Cout, double* Cfout, hipStream_t s) {
  using Dm = Dims<K>;
  if (!Cout) {
    const size_t tot = (size_t)mesh->nfc * Dm::D2 * Dm::D2;
    k_zero_diag<Dm::D2><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(mesh->d_diag, (int)mesh->nfc, H, F);
    HDG_CHECK_LAUNCH("k_zero_diag");
  }
  if (n == 0) return HDG_OK;
  const hdg_tile_config lc = launch_config(K);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)lc.workgroups_per_cu * device_cu_count()));
  const hdg_mesh& m = *mesh;
  const Tables& tb = disc->dev;
  const int rm = lc.xcd_remap;
  if (Cout) {  // export form: one shape is enough
    k_condense<K, 256, true><<<grid, 256, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout, rm);
  } else {
    switch (lc.waves_per_element) {
      case 1: k_condense<K, 64, false><<<grid, 64, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout, rm); break;
      case 2: k_condense<K, 128, false><<<grid, 128, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout, rm); break;
      case 4: k_condense<K, 256, false><<<grid, 256, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout, rm); break;
      default: k_condense<K, 512, false><<<grid, 512, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout, rm); break;
    }
  }
  HDG_CHECK_LAUNCH("k_condense");
  return HDG_OK;
}

}  // namespace

hdg_status dispatch_condense_tile(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                                  const double* f, const double* tau, double* H, double* F, double* factors,
                                  const int* elems, int64_t n, double* Cout, double* Cfout, double* dws,
                                  hipStream_t s);

namespace {

hdg_status dispatch_condense(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                             const double* f, const double* tau, double* H, double* F, double* factors,
                             const int* elems, int64_t n, double* Cout, double* Cfout, hipStream_t s,
                             double* dws = nullptr) {
  if (disc->host.k >= 1 && disc->host.k <= 3)
    return dispatch_condense_tile(disc, mesh, kappa, c, f, tau, H, F, factors, elems, n, Cout, Cfout, dws, s);
  switch (disc->host.k) {
    case 0: return run_condense<0>(disc, mesh, kappa, c, f, tau, H, F, factors, elems, n, Cout, Cfout, s);
    case 4: return run_condense<4>(disc, mesh, kappa, c, f, tau, H, F, factors, elems, n, Cout, Cfout, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "unsupported degree");
}

}  // namespace

hdg_status launch_batch_condense_tile(int k, const Tables& tb, const BatchItem* d_items, int nitems, int total_units,
                                      int grid, int xcd_remap, hipStream_t s);

int condense_unit(int k) { return (k >= 1 && k <= 3) ? 4 : 1; }

namespace {

template <int K>
hdg_status launch_batch_element(const Tables& tb, const BatchItem* d_items, int nitems, int total_units, int grid,
                                int xcd_remap, int waves, hipStream_t s) {
  switch (waves) {
    case 1: k_batch_condense<K, 64><<<grid, 64, 0, s>>>(d_items, nitems, total_units, tb, xcd_remap); break;
    case 2: k_batch_condense<K, 128><<<grid, 128, 0, s>>>(d_items, nitems, total_units, tb, xcd_remap); break;
    case 4: k_batch_condense<K, 256><<<grid, 256, 0, s>>>(d_items, nitems, total_units, tb, xcd_remap); break;
    case 8: k_batch_condense<K, 512><<<grid, 512, 0, s>>>(d_items, nitems, total_units, tb, xcd_remap); break;
    default: return set_error(HDG_ERR_INVALID_ARG, "batched condensation: waves_per_element must be 1, 2, 4 or 8");
  }
  HDG_CHECK_LAUNCH("k_batch_condense");
  return HDG_OK;
}

}  // namespace

hdg_status launch_batch_condense(int k, const Tables& tb, const BatchItem* d_items, int nitems, int total_units,
                                 int grid, int xcd_remap, int waves, hipStream_t s) {
  if (nitems <= 0 || total_units <= 0) return HDG_OK;
  if (k >= 1 && k <= 3) return launch_batch_condense_tile(k, tb, d_items, nitems, total_units, grid, xcd_remap, s);
  switch (k) {
    case 0: return launch_batch_element<0>(tb, d_items, nitems, total_units, grid, xcd_remap, waves, s);
    case 4: return launch_batch_element<4>(tb, d_items, nitems, total_units, grid, xcd_remap, waves, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "batched condensation: unsupported degree");
}

hdg_status check_disc_mesh(const hdg_disc* disc, const hdg_mesh* mesh, const char* who) {
  if (!disc || !mesh) return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": NULL handle");
  if (disc->host.nq != disc->host.k + 2)
    return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": compute kernels are built for nq = k + 2 only");
  if (mesh->nelt < 1 || mesh->nfc < 1 || !mesh->d_coords || !mesh->d_elements || !mesh->d_facebyele ||
      !mesh->d_perm || !mesh->d_normals || !mesh->d_slot || !mesh->d_diag)
    return set_error(HDG_ERR_INVALID_ARG, std::string(who) + ": mesh is not expanded");
  return HDG_OK;
}

}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_assemble_condense(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                            const double* d_c, const double* d_f, const double* d_tau, double* d_H,
                                            double* d_F, double* d_factors, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_assemble_condense");
  if (st) return st;
  if (!d_kappa || !d_c || !d_f || !d_tau || !d_H || !d_F)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_assemble_condense: NULL array");
  return dispatch_condense(disc, mesh, d_kappa, d_c, d_f, d_tau, d_H, d_F, d_factors, nullptr, mesh->nelt, nullptr,
                           nullptr, (hipStream_t)stream);
}

extern "C" hdg_status hdg_condense_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, size_t* bytes) {
  if (!disc || !mesh || !bytes) return set_error(HDG_ERR_INVALID_ARG, "hdg_condense_workspace_size: NULL argument");
  *bytes = (disc->host.k >= 1 && disc->host.k <= 3) ? condense_ws_bytes(disc->host.d2, mesh->nelt) : 0;
  return HDG_OK;
}

extern "C" hdg_status hdg_assemble_condense_ws(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                               const double* d_c, const double* d_f, const double* d_tau,
                                               double* d_H, double* d_F, double* d_factors, void* d_ws,
                                               size_t ws_bytes, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_assemble_condense_ws");
  if (st) return st;
  if (!d_kappa || !d_c || !d_f || !d_tau || !d_H || !d_F || !mesh->d_face_elem)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_assemble_condense_ws: NULL array");
  size_t need = 0;
  hdg_condense_workspace_size(disc, mesh, &need);
  if (need && (!d_ws || ws_bytes < need))
    return set_error(HDG_ERR_WORKSPACE, "hdg_assemble_condense_ws: workspace too small");
  return dispatch_condense(disc, mesh, d_kappa, d_c, d_f, d_tau, d_H, d_F, d_factors, nullptr, mesh->nelt, nullptr,
                           nullptr, (hipStream_t)stream, need ? (double*)d_ws : nullptr);
}

extern "C" hdg_status hdg_export_local(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                       const double* d_c, const double* d_f, const double* d_tau,
                                       const int32_t* d_elems, int64_t n, double* d_C, double* d_Cf, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_export_local");
  if (st) return st;
  if (!d_kappa || !d_c || !d_f || !d_tau || !d_elems || !d_C || !d_Cf || n < 0)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_export_local: NULL array");
  return dispatch_condense(disc, mesh, d_kappa, d_c, d_f, d_tau, nullptr, nullptr, nullptr, d_elems, n, d_C, d_Cf,
                           (hipStream_t)stream);
}
