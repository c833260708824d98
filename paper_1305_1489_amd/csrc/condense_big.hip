// Degrees 5 and 6: assembly, static condensation and scatter (Sections 3-6, eq 5.1-5.6),
// and the local postprocess u* (eq 9.11), for element blocks too large for LDS.
//
// The mathematics is that of the per-element kernel of degrees 0 and 4 (block elimination of
// q with A1 symmetric up to the sign of its last block row):
//   L L^T = M;  W_s = L^{-1} C_s^T;  S = Mc + tauPP + sum_s W_s^T W_s = Ls Ls^T;
//   Z_l = L^{-1} DP_l^T;  B_l = T_l DP_l^T + (sum_s n_{l s} W_s)^T Z_l;  V = Ls^{-1} [B | f];
//   C^K = tauDD + [ (n_l . n_m) Z_l^T Z_m ]_{lm} - V^T V,   Cf^K = V^T Ls^{-1} f,
// with the same factor store (L, Ls packed lower, f), so the per-element reconstruction reads
// it unchanged.  At k = 6 (d3 = 84, 4 d2 = 112) the solved blocks W | Z and B | f take
// 40 k doubles (313 KB) per element: one workgroup takes one element at a time and keeps
// the two d3 x d3 factors, the point weights and a chunk of the basis table in LDS
// (149 KB at k = 6, 74 KB at k = 5), and the solved blocks in its own slice of a caller
// workspace (global memory, resident in the L2 and last-level caches while the element is
// worked on).  Phases:
//   Gram sums: the basis table streamed through LDS in chunks of points, one tile of M and
//     Mc per thread over the upper triangle (2 x 4 at k = 5, 4 x 4 at k = 6);
//   factorisations: the leading 64 rows by one wavefront with its rows in registers, the
//     rest (k = 6) by a block step (U12 = L11^{-1} A12, A22 -= U12^T U12, factor A22);
//   triangular solves: one right-hand side per thread in registers;
//   products S, B and C^K: their operands (W_s; U_l = sum_s n_{l s} W_s with Z_l; the Z and
//     V blocks of a face pair) staged in LDS over the factors once these are used up, 4 x 4
//     (S, B) or 2 x 2 (C^K) register tiles per thread.
#include "device_common.h"
#include "tile.h"

namespace hdg {
namespace {

constexpr int kBigThreads = 256;
// Threads of the condensation workgroup: six wavefronts at k = 6, so that the 364
// right-hand sides of the first triangular solve take one round (one per thread), four at
// k = 5 (252 of them).
constexpr int cond_threads(int k) { return k == 6 ? 384 : 256; }

template <int K>
struct BigDims {
  static constexpr int D3 = dim3(K), D2 = dim2(K), M = 4 * D2, NQD = (K + 2) * (K + 2) * (K + 2);
  static constexpr int D3P = dim3(K + 1);
  static constexpr int NCOL = 3 * D3 + M;  // right-hand sides C_s^T, then DP_l^T
  static constexpr int NV = M + 1;         // B and f, then V = Ls^{-1} [B | f]
  static constexpr int SLICE = D3 * NCOL + D3 * NV;  // workspace doubles per workgroup
  static constexpr int QC = 32;            // points per staged chunk of the basis table
  static constexpr int NTRI = D3 * (D3 + 1) / 2;
  static_assert(D3 % 4 == 0 && M % 4 == 0, "whole 4 x 4 tiles");
  static_assert(NCOL % 2 == 0 && (3 * D3) % 2 == 0, "16-byte pairs of the solved blocks");
};

// LDS of one element.  R holds, in order: U (M, then U = L^T), a chunk of the basis table,
// the point weights |K| w_q / kappa_q, |K| w_q c_q, |K| w_q f_q (NQDP each), and Us (Mc, then
// S, then Us = Ls^T).  Once L is used up, the space before Us stages the operands of the
// products S and B; once V is formed, the whole of R stages those of C^K.
template <int K>
struct BigSmem {
  using B = BigDims<K>;
  static constexpr int NQDP = B::NQD + (B::NQD & 1);
  static constexpr int OFF_PC = B::D3 * B::D3, OFF_W = OFF_PC + B::QC * B::D3, OFF_US = OFF_W + 3 * NQDP;
  static constexpr int LEN = OFF_US + B::D3 * B::D3;
  static constexpr int ZLD = (B::D2 + 3) / 4 * 4;  // face columns padded to whole tiles
  static_assert(OFF_US % 2 == 0, "16-byte rows of Us");
  static_assert(B::D3 * B::D3 + B::D3 * ZLD <= OFF_US, "U_l and Z_l fit before Us");
  static_assert(4 * B::D3 * ZLD <= LEN, "Z_l, Z_m, V_l, V_m fit in R");
  double R[LEN];
  double fv[B::D3], idl[B::D3], ids[B::D3];
  double nn[4][4];
  int slot[16], fbe[4];
};
static_assert(sizeof(BigSmem<6>) + sizeof(ElemGeom) <= 160 * 1024, "degree-6 LDS budget");

// Lower-triangle pair (i >= j) of index p in row-major order: p = i (i + 1) / 2 + j.
__device__ __forceinline__ void lower_pair(int p, int& i, int& j) {
  int r = (int)((sqrtf(8.0f * p + 1.0f) - 1.0f) * 0.5f);
  while (r * (r + 1) / 2 > p) --r;
  while ((r + 1) * (r + 2) / 2 <= p) ++r;
  i = r;
  j = p - r * (r + 1) / 2;
}

// x <- U^{-T} x (forward substitution with L = U^T, rows of U with leading dimension LD) for
// one right-hand side in registers; every thread reads the same LDS words.
template <int N, int LD = N>
__device__ __forceinline__ void reg_forward(const double* U, const double* idg, double (&x)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double xk = x[k] * idg[k];
    x[k] = xk;
#pragma unroll
    for (int r = k + 1; r < N; ++r) x[r] = fma(-U[k * LD + r], xk, x[r]);
    __builtin_amdgcn_sched_barrier(0);  // one row of LDS reads in flight at a time
  }
}

// Copy of n items by the workgroup, eight global loads in flight per thread before their
// LDS stores: ld(i) reads item i, st(i, v) stores it.
template <int NT, class Ld, class St>
__device__ __forceinline__ void stage_batched(int n, int t, Ld ld, St st) {
  for (int b = t; b < n; b += 8 * NT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = b + u * NT;
      v[u] = i < n ? ld(i) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = b + u * NT;
      if (i < n) st(i, v[u]);
    }
  }
}

// The same factorisation right-looking over the whole workgroup: step k updates the
// trailing upper triangle (its entries spread over all threads) with the unscaled row k
// divided by its pivot and scales row k - 1, which no thread reads any more, so each step
// needs one barrier.  Used where it measured faster (the degree-6 stiffness matrix of the
// degree-5 postprocess, which runs at two workgroups per CU).
template <int N>
__device__ inline void lds_chol_rows(double* A, double* idg) {
  const int t = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < N; ++k) {
    __syncthreads();
    if (k > 0) {
      const int kp = k - 1;
      const double is = idg[kp];
      for (int c = kp + t; c < N; c += nt) A[kp * N + c] *= is;
    }
    const double d = A[k * N + k];
    if (t == 0) idg[k] = 1.0 / sqrt(d);
    const double rd = 1.0 / d;
    const int nr = N - k - 1;
    for (int idx = t; idx < nr * nr; idx += nt) {
      const int i = k + 1 + idx / nr, j = k + 1 + idx % nr;
      if (j >= i) A[i * N + j] -= A[k * N + i] * A[k * N + j] * rd;
    }
  }
  __syncthreads();
  if (t == 0) A[(N - 1) * N + N - 1] *= idg[N - 1];
  __syncthreads();
}

// In-place Cholesky factorisation A = U^T U of the N x N SPD matrix held in the upper
// triangle of A (row-major, entries (i, j) with i <= j), by the workgroup; idg receives
// 1 / U_kk.  The leading block of up to 64 rows is factored by one wavefront with its rows in
// registers (wave_cholesky); for N > 64 the trailing rows follow by blocks:
// U12 = L11^{-1} A12 (one column per thread), A22 -= U12^T U12, and the one-wavefront
// factorisation of A22.
template <int N>
__device__ inline void lds_chol_upper(double* A, double* idg) {
  constexpr int N1 = N <= 64 ? N : 64, N2 = N - N1;
  static_assert(N2 <= 64, "two diagonal blocks");
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  __syncthreads();
  if (wave == 0) {
    const double* const parts[1] = {A};
    wave_cholesky<N1, N, 1>(parts, A, idg, lane);
  }
  __syncthreads();
  if constexpr (N2 > 0) {
    if (t < N2) {
      const int i = N1 + t;
      double x[N1];
#pragma unroll
      for (int r = 0; r < N1; ++r) x[r] = A[r * N + i];
      reg_forward<N1, N>(A, idg, x);
#pragma unroll
      for (int r = 0; r < N1; ++r) A[r * N + i] = x[r];
    }
    __syncthreads();
    for (int p = t; p < N2 * N2; p += blockDim.x) {
      const int i = N1 + p / N2, j = N1 + p % N2;
      if (j < i) continue;
      double sacc = 0;
      for (int r = 0; r < N1; ++r) sacc = fma(A[r * N + i], A[r * N + j], sacc);
      A[i * N + j] -= sacc;
    }
    __syncthreads();
    if (wave == 0) {
      const double* const parts[1] = {A + N1 * N + N1};
      wave_cholesky<N2, N, 1>(parts, A + N1 * N + N1, idg + N1, lane);
    }
    __syncthreads();
  }
}

template <int K, bool EXPORT>
__global__ void __launch_bounds__(cond_threads(K)) k_condense_big(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                              const double* __restrict__ cco,
                                                              const double* __restrict__ fco,
                                                              const double* __restrict__ tau, double* __restrict__ H,
                                                              double* __restrict__ F, double* __restrict__ factors,
                                                              const int* __restrict__ elems, int nwork,
                                                              double* __restrict__ Cout, double* __restrict__ Cfout,
                                                              double* __restrict__ ws, int xcd_remap) {
  using B = BigDims<K>;
  constexpr int D3 = B::D3, D2 = B::D2, M = B::M, NQD = B::NQD, NCOL = B::NCOL, NV = B::NV, QC = B::QC;
  constexpr int NTRI = B::NTRI, NT = cond_threads(K);
  constexpr int TT = D3 / 4, ZLD = BigSmem<K>::ZLD, NQDP = BigSmem<K>::NQDP;
  constexpr int GRAM_ROWS = K == 5 ? 2 : 4;
  constexpr int GJOBS = GRAM_ROWS == 4 ? TT * (TT + 1) / 2 : TT * (TT + 1);
  static_assert(GJOBS <= NT, "one Gram tile per thread");
  static_assert(TT * (TT + 1) / 2 <= NT && TT * (ZLD / 4) <= NT && (ZLD / 2) * (ZLD / 2) <= NT,
                "one product tile per thread");
  __shared__ __align__(16) BigSmem<K> sm;
  __shared__ ElemGeom sg;
  double* R = sm.R;
  double* U = R;
  double* Pc = R + BigSmem<K>::OFF_PC;
  double* wk = R + BigSmem<K>::OFF_W;
  double* wc = wk + NQDP;
  double* wf = wc + NQDP;
  double* Us = R + BigSmem<K>::OFF_US;
  double* X = ws + (size_t)blockIdx.x * B::SLICE;  // [D3][NCOL]: W_0 | W_1 | W_2 | Z
  double* Vb = X + (size_t)D3 * NCOL;              // [D3][NV]:   B | f, then V
  for (int w = batch_block(xcd_remap); w < nwork; w += gridDim.x) {
    // the thread index passes through an opaque move, so the per-thread addresses derived
    // from it are formed where they are used, not hoisted out of the element loop (where
    // they would stay live across every phase and spill)
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int E = EXPORT ? elems[w] : w;
    if (E < 0 || E >= mesh.nelt) continue;  // uniform across the workgroup
    // ---- geometry, scatter slots and the point weights (eq 3.5)
    if (t == 0) load_geometry(E, mesh, tau, sg);
    if (t < 16) sm.slot[t] = mesh.d_slot[16 * E + t];
    if (t < 4) sm.fbe[t] = mesh.d_facebyele[4 * E + t];
    __syncthreads();
    for (int q = t; q < NQD; q += NT) {
      const double wq = sg.vol * tb.vol_w[q];
      wk[q] = wq / kappa[(size_t)E * NQD + q];
      wc[q] = wq * cco[(size_t)E * NQD + q];
      wf[q] = wq * fco[(size_t)E * NQD + q];
    }
    if (t < 16) {
      const int l = t / 4, m = t % 4;
      sm.nn[l][m] = sg.n[l][0] * sg.n[m][0] + sg.n[l][1] * sg.n[m][1] + sg.n[l][2] * sg.n[m][2];
    }
    // ---- M = P^T diag(|K| w / kappa) P, Mc = P^T diag(|K| w c) P, f = P^T (|K| w f) (eq 3.5,
    // eq 4.5), the basis table streamed through LDS in chunks of QC points, one GR x 4 tile
    // of both matrices per thread over the upper triangle: rows GR gi .. GR gi + GR - 1,
    // columns 4 gj .. 4 gj + 3 (GR = 2 at k = 5, so that 210 threads share the work, 4 at k = 6)
    constexpr int GR = GRAM_ROWS;
    const bool gjob = t < GJOBS;
    int gi = 0, gj = 0;
    if (gjob) {
      if constexpr (GR == 4) {
        lower_pair(t, gj, gi);
      } else {  // column tile gj holds 2 gj + 2 row pairs: job p = gj (gj + 1) + gi
        gj = (int)((sqrtf(4.0f * t + 1.0f) - 1.0f) * 0.5f);
        while (gj * (gj + 1) > t) --gj;
        while ((gj + 1) * (gj + 2) <= t) ++gj;
        gi = t - gj * (gj + 1);
      }
    }
    double am[GR][4] = {}, ac[GR][4] = {}, ff = 0;
    for (int q0 = 0; q0 < NQD; q0 += QC) {
      const int nq = min(QC, NQD - q0);
      __syncthreads();
      const double* pchunk = tb.P + (size_t)q0 * D3;
      stage_batched<NT>(nq * D3, t, [&](int i) { return pchunk[i]; }, [&](int i, double v) { Pc[i] = v; });
      __syncthreads();
      if (gjob) {
        for (int q = 0; q < nq; ++q) {
          const double* pq = Pc + q * D3;
          double av[GR];
#pragma unroll
          for (int a = 0; a < GR; a += 2) {
            const double2 v = *reinterpret_cast<const double2*>(pq + GR * gi + a);
            av[a] = v.x;
            av[a + 1] = v.y;
          }
          const double2 b01 = *reinterpret_cast<const double2*>(pq + 4 * gj);
          const double2 b23 = *reinterpret_cast<const double2*>(pq + 4 * gj + 2);
          const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
          const double wkq = wk[q0 + q], wcq = wc[q0 + q];
#pragma unroll
          for (int a = 0; a < GR; ++a) {
            const double ka = wkq * av[a], ca = wcq * av[a];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              am[a][b] = fma(ka, bv[b], am[a][b]);
              ac[a][b] = fma(ca, bv[b], ac[a][b]);
            }
          }
        }
      }
      if (t < D3)
        for (int q = 0; q < nq; ++q) ff = fma(wf[q0 + q], Pc[q * D3 + t], ff);
    }
    if (gjob) {
#pragma unroll
      for (int a = 0; a < GR; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = GR * gi + a, j = 4 * gj + b;
          if (i <= j) {
            U[i * D3 + j] = am[a][b];
            Us[i * D3 + j] = ac[a][b];
          }
        }
    }
    if (t < D3) sm.fv[t] = ff;
    // ---- L (eq 5.1), stored packed for the reconstruction
    lds_chol_upper<D3>(U, sm.idl);
    double* fa = (!EXPORT && factors) ? factors + (size_t)E * (D3 * (D3 + 1) + D3) : nullptr;
    if (fa) {
      for (int p = t; p < NTRI; p += NT) {
        int i, j;
        lower_pair(p, i, j);
        fa[p] = U[j * D3 + i];  // L[i][j] = U[j][i]
      }
      if (t < D3) fa[D3 * (D3 + 1) + t] = sm.fv[t];
    }
    // ---- W_s = L^{-1} C_s^T and Z_l = L^{-1} DP_l^T (eq 5.2): column c < 3 D3 is (s, i),
    // its right-hand side sum_h a[s][h] Chat[h][i][.]; the others are (l, i), DP[mu_l][l][i][.]
    for (int c = t; c < NCOL; c += NT) {
      double x[D3];
      if (c < 3 * D3) {
        const int s = c / D3, i = c % D3;
        const double a0 = sg.a[s][0], a1 = sg.a[s][1], a2 = sg.a[s][2];
        const double* c0 = tb.Chat + (size_t)i * D3;
#pragma unroll
        for (int r = 0; r < D3; ++r)
          x[r] = a0 * c0[r] + a1 * c0[(size_t)D3 * D3 + r] + a2 * c0[(size_t)2 * D3 * D3 + r];
      } else {
        const int l = (c - 3 * D3) / D2, i = (c - 3 * D3) % D2;
        const double* dp = tb.DP + ((size_t)(sg.mu[l] * 4 + l) * D2 + i) * D3;
#pragma unroll
        for (int r = 0; r < D3; ++r) x[r] = dp[r];
      }
      reg_forward<D3>(U, sm.idl, x);
#pragma unroll
      for (int r = 0; r < D3; ++r) X[(size_t)r * NCOL + c] = x[r];
    }
    __syncthreads();
    // ---- S = Mc + sum_l T_l PP_l + sum_s W_s^T W_s (eq 5.3) on the upper 4 x 4 tiles (at
    // most one per thread), each W_s staged in LDS over L, which is no longer needed
    {
      const bool job = t < TT * (TT + 1) / 2;
      int ti = 0, tj = 0;  // ti <= tj
      if (job) lower_pair(t, tj, ti);
      double acc[4][4] = {};
      for (int s = 0; s < 3; ++s) {
        __syncthreads();
        for (int idx = t; idx < D3 * D3 / 2; idx += NT) {
          const int r = 2 * idx / D3, i = 2 * idx % D3;
          *reinterpret_cast<double2*>(R + r * D3 + i) =
              *reinterpret_cast<const double2*>(X + (size_t)r * NCOL + s * D3 + i);
        }
        __syncthreads();
        if (job) {
#pragma unroll 4
          for (int r = 0; r < D3; ++r) {
            const double2 a01 = *reinterpret_cast<const double2*>(R + r * D3 + 4 * ti);
            const double2 a23 = *reinterpret_cast<const double2*>(R + r * D3 + 4 * ti + 2);
            const double2 b01 = *reinterpret_cast<const double2*>(R + r * D3 + 4 * tj);
            const double2 b23 = *reinterpret_cast<const double2*>(R + r * D3 + 4 * tj + 2);
            const double av[4] = {a01.x, a01.y, a23.x, a23.y}, bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
          }
        }
      }
      if (job) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int i = 4 * ti + a, j = 4 * tj + b;
            if (i > j) continue;
            double v = Us[i * D3 + j] + acc[a][b];
#pragma unroll
            for (int l = 0; l < 4; ++l) v = fma(sg.T[l], tb.PP[((size_t)l * D3 + i) * D3 + j], v);
            Us[i * D3 + j] = v;
          }
      }
    }
    // ---- Ls (eq 5.4), stored packed after L, then f
    lds_chol_upper<D3>(Us, sm.ids);
    if (fa) {
      for (int p = t; p < NTRI; p += NT) {
        int i, j;
        lower_pair(p, i, j);
        fa[NTRI + p] = Us[j * D3 + i];
      }
    }
    // ---- B_l = T_l DP_l^T + U_l^T Z_l with U_l = sum_s n_{l s} W_s (eq 5.2), face by face:
    // U_l and Z_l (its columns padded to ZLD with zeros) staged in LDS, one 4 x 4 tile of
    // (rows i of the u space, columns of face l) per thread; then the f column
    for (int l = 0; l < 4; ++l) {
      __syncthreads();
      double* Ul = R;
      double* Zl = R + D3 * D3;
      const double n0 = sg.n[l][0], n1 = sg.n[l][1], n2 = sg.n[l][2];
      for (int idx = t; idx < D3 * D3 / 2; idx += NT) {
        const int r = 2 * idx / D3, i = 2 * idx % D3;
        const double* xr = X + (size_t)r * NCOL + i;
        const double2 w0 = *reinterpret_cast<const double2*>(xr);
        const double2 w1 = *reinterpret_cast<const double2*>(xr + D3);
        const double2 w2 = *reinterpret_cast<const double2*>(xr + 2 * D3);
        *reinterpret_cast<double2*>(Ul + r * D3 + i) =
            make_double2(n0 * w0.x + n1 * w1.x + n2 * w2.x, n0 * w0.y + n1 * w1.y + n2 * w2.y);
      }
      for (int idx = t; idx < D3 * ZLD; idx += NT) {
        const int r = idx / ZLD, c = idx % ZLD;
        Zl[idx] = c < D2 ? X[(size_t)r * NCOL + 3 * D3 + l * D2 + c] : 0.0;
      }
      __syncthreads();
      if (t < TT * (ZLD / 4)) {
        const int ti = t / (ZLD / 4), tc = t % (ZLD / 4);
        double acc[4][4] = {};
#pragma unroll 4
        for (int r = 0; r < D3; ++r) {
          const double2 a01 = *reinterpret_cast<const double2*>(Ul + r * D3 + 4 * ti);
          const double2 a23 = *reinterpret_cast<const double2*>(Ul + r * D3 + 4 * ti + 2);
          const double2 b01 = *reinterpret_cast<const double2*>(Zl + r * ZLD + 4 * tc);
          const double2 b23 = *reinterpret_cast<const double2*>(Zl + r * ZLD + 4 * tc + 2);
          const double av[4] = {a01.x, a01.y, a23.x, a23.y}, bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int ia = 4 * tc + b;
          if (ia >= D2) continue;
          const double* dp = tb.DP + ((size_t)(sg.mu[l] * 4 + l) * D2 + ia) * D3;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int i = 4 * ti + a;
            Vb[(size_t)i * NV + l * D2 + ia] = fma(sg.T[l], dp[i], acc[a][b]);
          }
        }
      }
    }
    if (t < D3) Vb[(size_t)t * NV + M] = sm.fv[t];
    __syncthreads();
    // ---- V = Ls^{-1} [B | f], one column per thread
    for (int c = t; c < NV; c += NT) {
      double x[D3];
#pragma unroll
      for (int r = 0; r < D3; ++r) x[r] = Vb[(size_t)r * NV + c];
      reg_forward<D3>(Us, sm.ids, x);
#pragma unroll
      for (int r = 0; r < D3; ++r) Vb[(size_t)r * NV + c] = x[r];
    }
    __syncthreads();
    // ---- C^K = tauDD + (n_l . n_m) Z_l^T Z_m - V^T V (eq 5.6) by face pairs l <= m: Z_l,
    // Z_m, V_l, V_m staged in LDS (columns padded to ZLD with zeros; the factors are dead),
    // one 2 x 2 tile per thread; scattered (eq 6.5: off-diagonal blocks have one writer,
    // diagonal blocks two addends onto zeros) or exported.  Then Cf^K = V^T Ls^{-1} f.
    for (int l = 0; l < 4; ++l)
      for (int m = l; m < 4; ++m) {
        __syncthreads();
        double* Za = R;
        double* Zb = R + D3 * ZLD;
        double* Va = R + 2 * D3 * ZLD;
        double* Vc = R + 3 * D3 * ZLD;
        // item e of the four blocks: block e / (D3 ZLD), row, padded column
        stage_batched<NT>(
            4 * D3 * ZLD, t,
            [&](int e) {
              const int blk = e / (D3 * ZLD), rc = e % (D3 * ZLD), r = rc / ZLD, c = rc % ZLD;
              const int col = (blk & 1 ? m : l) * D2 + c;
              const double* src = blk < 2 ? X + (size_t)r * NCOL + 3 * D3 : Vb + (size_t)r * NV;
              return c < D2 ? src[col] : 0.0;
            },
            [&](int e, double v) { R[e] = v; });
        __syncthreads();
        constexpr int T2 = ZLD / 2;
        if (t < T2 * T2) {
          const int ta = t / T2, tb2 = t % T2;
          if (l < m || ta <= tb2) {
            double az[2][2] = {}, av[2][2] = {};
#pragma unroll 4
            for (int r = 0; r < D3; ++r) {
              const double2 za = *reinterpret_cast<const double2*>(Za + r * ZLD + 2 * ta);
              const double2 zb = *reinterpret_cast<const double2*>(Zb + r * ZLD + 2 * tb2);
              const double2 va = *reinterpret_cast<const double2*>(Va + r * ZLD + 2 * ta);
              const double2 vb = *reinterpret_cast<const double2*>(Vc + r * ZLD + 2 * tb2);
              az[0][0] = fma(za.x, zb.x, az[0][0]);
              az[0][1] = fma(za.x, zb.y, az[0][1]);
              az[1][0] = fma(za.y, zb.x, az[1][0]);
              az[1][1] = fma(za.y, zb.y, az[1][1]);
              av[0][0] = fma(va.x, vb.x, av[0][0]);
              av[0][1] = fma(va.x, vb.y, av[0][1]);
              av[1][0] = fma(va.y, vb.x, av[1][0]);
              av[1][1] = fma(va.y, vb.y, av[1][1]);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
              for (int b = 0; b < 2; ++b) {
                const int ia = 2 * ta + a, ib = 2 * tb2 + b;
                if (ia >= D2 || ib >= D2 || (l == m && ia > ib)) continue;
                const int ra = l * D2 + ia, cb = m * D2 + ib;
                double v = sm.nn[l][m] * az[a][b] - av[a][b];
                if (ra == cb) v += sg.T[l];
                if (EXPORT) {
                  Cout[((size_t)w * M + ra) * M + cb] = v;
                  Cout[((size_t)w * M + cb) * M + ra] = v;
                } else {
                  const size_t s1 = sm.slot[4 * l + m];
                  if (l == m) {
                    unsafeAtomicAdd(&H[(s1 * D2 + ia) * D2 + ib], v);
                    if (ia != ib) unsafeAtomicAdd(&H[(s1 * D2 + ib) * D2 + ia], v);
                  } else {
                    const size_t s2 = sm.slot[4 * m + l];
                    H[(s1 * D2 + ia) * D2 + ib] = v;
                    H[(s2 * D2 + ib) * D2 + ia] = v;
                  }
                }
              }
          }
        }
      }
    for (int a = t; a < M; a += NT) {
      double v = 0;
      for (int r = 0; r < D3; ++r) v = fma(Vb[(size_t)r * NV + a], Vb[(size_t)r * NV + M], v);
      if (EXPORT)
        Cfout[(size_t)w * M + a] = v;
      else
        unsafeAtomicAdd(&F[(size_t)sm.fbe[a / D2] * D2 + a % D2], v);
    }
    __syncthreads();  // LDS and the workspace slice are reused by the next element
  }
}

// Zero the diagonal blocks of H and F before the scatter.
template <int D2>
__global__ void k_zero_diag_big(const int* __restrict__ diag, int nfc, double* __restrict__ H, double* __restrict__ F) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)nfc * D2 * D2) return;
  const size_t f = i / (D2 * D2), e = i % (D2 * D2);
  H[(size_t)diag[f] * D2 * D2 + e] = 0.0;
  if (e < D2) F[f * D2 + e] = 0.0;
}

// ---- local postprocess u* (eq 9.11), one element per workgroup.  With V = Q a (Q the
// recovered flux coefficients, a the cofactor matrix), for each point q
//   Y_h(q) = |K| w_q / (kappa_q det) sum_j P_j(p_q) V[j][h],
//   rhs_i  = -sum_h sum_q Y_h(q) gradhat_h P_i(p_q)   (i >= 1),   rhs_0 = u_0,
//   S*_ij  = sum_{h <= g} G_hg Shat^{hg}_ij with G = a^T a / det, identity on mode 0;
// S* is factored in LDS and the two triangular solves run over the workgroup.
template <int K>
struct PPBig {
  static constexpr int D3 = dim3(K), D3P = dim3(K + 1), NQD = (K + 2) * (K + 2) * (K + 2);
};

template <int K>
__global__ void __launch_bounds__(kBigThreads) k_pp_big(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                        const double* __restrict__ tau, const double* __restrict__ qin,
                                                        const double* __restrict__ uin, double* __restrict__ us) {
  using P = PPBig<K>;
  constexpr int D3 = P::D3, D3P = P::D3P, NQD = P::NQD, NT = kBigThreads;
  __shared__ double S[D3P * D3P];
  __shared__ double V[3 * D3], Y[3 * NQD], rhs[D3P], idg[D3P], part[kBigThreads];
  __shared__ ElemGeom g;
  const int t = threadIdx.x;
  for (int E = blockIdx.x; E < mesh.nelt; E += gridDim.x) {
    if (t == 0) load_geometry(E, mesh, tau, g);
    __syncthreads();
    for (int idx = t; idx < 3 * D3; idx += NT) {
      const int h = idx / D3, j = idx % D3;
      const double* qe = qin + (size_t)E * 3 * D3 + j;
      V[idx] = qe[0] * g.a[0][h] + qe[D3] * g.a[1][h] + qe[2 * D3] * g.a[2][h];
    }
    const double idet = 1.0 / g.det;
    double G[3][3];
#pragma unroll
    for (int h = 0; h < 3; ++h)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        G[h][k] = (g.a[0][h] * g.a[0][k] + g.a[1][h] * g.a[1][k] + g.a[2][h] * g.a[2][k]) * idet;
    const double cf[6] = {G[0][0], G[1][1], G[2][2], G[0][1], G[0][2], G[1][2]};
    for (int idx = t; idx < D3P * D3P; idx += NT) {
      const int i = idx / D3P, j = idx % D3P;
      double s = 0;
      if (i == 0 || j == 0) {
        s = i == j ? 1.0 : 0.0;
      } else {
#pragma unroll
        for (int p = 0; p < 6; ++p) s += cf[p] * tb.Shat[((size_t)p * D3P + i) * D3P + j];
      }
      S[idx] = s;
    }
    __syncthreads();
    const double wscale = g.vol / g.det;
    for (int q = t; q < NQD; q += NT) {
      const double wr = wscale * tb.vol_w[q] / kappa[(size_t)E * NQD + q];
      const double* pq = tb.P + (size_t)q * D3;
      double y0 = 0, y1 = 0, y2 = 0;
      for (int j = 0; j < D3; ++j) {
        const double p = pq[j];
        y0 = fma(p, V[j], y0);
        y1 = fma(p, V[D3 + j], y1);
        y2 = fma(p, V[2 * D3 + j], y2);
      }
      Y[q] = wr * y0;
      Y[NQD + q] = wr * y1;
      Y[2 * NQD + q] = wr * y2;
    }
    __syncthreads();
    {  // the gradient contraction over the (direction, point) pairs: mode i by two threads
       // (one half of the points each), four chains per thread
      static_assert(NT == 256 && D3P <= 128, "two threads per mode");
      const int i = t & 127, hf = t >> 7;
      const int q0 = hf ? NQD / 2 : 0, q1 = hf ? NQD : NQD / 2;
      double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
      if (i > 0 && i < D3P) {
        for (int h = 0; h < 3; ++h) {
          const double* gp = tb.P1g + (size_t)h * NQD * D3P + i;
          const double* yh = Y + h * NQD;
          int q = q0;
          for (; q + 3 < q1; q += 4) {
            s0 = fma(gp[(size_t)q * D3P], yh[q], s0);
            s1 = fma(gp[(size_t)(q + 1) * D3P], yh[q + 1], s1);
            s2 = fma(gp[(size_t)(q + 2) * D3P], yh[q + 2], s2);
            s3 = fma(gp[(size_t)(q + 3) * D3P], yh[q + 3], s3);
          }
          for (; q < q1; ++q) s0 = fma(gp[(size_t)q * D3P], yh[q], s0);
        }
      }
      part[t] = (s0 + s1) + (s2 + s3);
      __syncthreads();
      if (t < D3P) rhs[t] = t == 0 ? uin[(size_t)E * D3] : -(part[t] + part[128 + t]);
    }
    // S* = U^T U, then U^T y = rhs and U x = y
    if constexpr (K == 5)
      lds_chol_rows<D3P>(S, idg);
    else
      lds_chol_upper<D3P>(S, idg);
    for (int k = 0; k < D3P; ++k) {
      const double xk = rhs[k] * idg[k];
      for (int r = k + 1 + t; r < D3P; r += NT) rhs[r] -= S[k * D3P + r] * xk;
      __syncthreads();
      if (t == 0) rhs[k] = xk;
      __syncthreads();
    }
    for (int k = D3P - 1; k >= 0; --k) {
      const double xk = rhs[k] * idg[k];
      for (int r = t; r < k; r += NT) rhs[r] -= S[r * D3P + k] * xk;
      __syncthreads();
      if (t == 0) rhs[k] = xk;
      __syncthreads();
    }
    for (int i = t; i < D3P; i += NT) us[(size_t)E * D3P + i] = rhs[i];
    __syncthreads();
  }
}

template <int K>
int big_grid(int64_t n) {
  const hdg_tile_config lc = launch_config(K);
  return (int)std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)lc.workgroups_per_cu * device_cu_count()));
}

template <int K>
hdg_status run_condense_big(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                            const double* f, const double* tau, double* H, double* F, double* factors,
                            const int* elems, int64_t n, double* Cout, double* Cfout, double* ws, size_t ws_bytes,
                            hipStream_t s) {
  using B = BigDims<K>;
  const int grid = big_grid<K>(n);
  if (!ws || ws_bytes < (size_t)grid * B::SLICE * sizeof(double))
    return set_error(HDG_ERR_WORKSPACE,
                     "degrees 5 and 6 keep the solved element blocks in a caller workspace "
                     "(hdg_condense_workspace_size bytes): use hdg_assemble_condense_ws");
  if (!Cout) {
    const size_t tot = (size_t)mesh->nfc * B::D2 * B::D2;
    k_zero_diag_big<B::D2><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(mesh->d_diag, (int)mesh->nfc, H, F);
    HDG_CHECK_LAUNCH("k_zero_diag_big");
  }
  if (n == 0) return HDG_OK;
  const int rm = launch_config(K).xcd_remap;
  if (Cout) {
    k_condense_big<K, true><<<grid, cond_threads(K), 0, s>>>(*mesh, disc->dev, kappa, c, f, tau, nullptr, nullptr,
                                                          nullptr, elems, (int)n, Cout, Cfout, ws, rm);
  } else {
    timer_begin("k_condense", s);
    k_condense_big<K, false><<<grid, cond_threads(K), 0, s>>>(*mesh, disc->dev, kappa, c, f, tau, H, F, factors,
                                                           nullptr, (int)n, nullptr, nullptr, ws, rm);
    timer_end("k_condense", s);
  }
  HDG_CHECK_LAUNCH("k_condense_big");
  return HDG_OK;
}

}  // namespace

size_t condense_big_workspace_bytes(int k, int64_t n) {
  switch (k) {
    case 5: return (size_t)big_grid<5>(n) * BigDims<5>::SLICE * sizeof(double);
    case 6: return (size_t)big_grid<6>(n) * BigDims<6>::SLICE * sizeof(double);
  }
  return 0;
}

hdg_status dispatch_condense_big(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                                 const double* f, const double* tau, double* H, double* F, double* factors,
                                 const int* elems, int64_t n, double* Cout, double* Cfout, double* ws,
                                 size_t ws_bytes, hipStream_t s) {
  switch (disc->host.k) {
    case 5: return run_condense_big<5>(disc, mesh, kappa, c, f, tau, H, F, factors, elems, n, Cout, Cfout, ws, ws_bytes, s);
    case 6: return run_condense_big<6>(disc, mesh, kappa, c, f, tau, H, F, factors, elems, n, Cout, Cfout, ws, ws_bytes, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "condensation: unsupported degree");
}

hdg_status launch_postprocess_big(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* tau,
                                  const double* q, const double* u, double* us, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(mesh->nelt, 2 * (int64_t)device_cu_count()));
  timer_begin("k_pp_big", s);
  switch (disc->host.k) {
    case 5: k_pp_big<5><<<grid, kBigThreads, 0, s>>>(*mesh, disc->dev, kappa, tau, q, u, us); break;
    case 6: k_pp_big<6><<<grid, kBigThreads, 0, s>>>(*mesh, disc->dev, kappa, tau, q, u, us); break;
    default: return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "postprocess: unsupported degree");
  }
  timer_end("k_pp_big", s);
  HDG_CHECK_LAUNCH("k_pp_big");
  return HDG_OK;
}

}  // namespace hdg
