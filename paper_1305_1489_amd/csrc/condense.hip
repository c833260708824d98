// Assembly of the element blocks, static condensation onto the four face traces, and
// scatter into the global trace system (Sections 3-6 of the paper).
//
// Per element K (degrees 0 and 4 here; 1..3 run as tiles of four elements elsewhere), on
// one workgroup with the blocks resident in LDS:
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
#include "tile.h"

namespace hdg {
namespace {

// Upper pair (i <= j) of an n x n matrix from its index p in the row-major order of the
// upper triangle (counted from the end, kk = r (r + 1) / 2 + s with r = n - 1 - i).
__device__ __forceinline__ void upper_pair(int p, int n, int& i, int& j) {
  const int kk = n * (n + 1) / 2 - 1 - p;
  int r = (int)((sqrtf(8.0f * kk + 1.0f) - 1.0f) * 0.5f);
  while (r * (r + 1) / 2 > kk) --r;
  while ((r + 1) * (r + 2) / 2 <= kk) ++r;
  i = n - 1 - r;
  j = n - 1 - (kk - r * (r + 1) / 2);
}

// x <- L^{-1} x for one right-hand side in registers, L given by Lt = L^T (leading
// dimension LD even, 16-byte aligned rows) and its reciprocal diagonal; column-oriented,
// so the updates of one pass are independent, and every lane reads the same LDS words.
template <int N, int LD>
__device__ __forceinline__ void col_forward(const double* Lt, const double* idg, double (&x)[N]) {
  // the leading PF pairs of row k + 1 are fetched during pass k (they are the first used
  // in pass k + 1), the rest of each row at the start of its own pass
  constexpr int NP = LD / 2, PF = 6;
  double2 nxt[PF];
  double dn = idg[0];
#pragma unroll
  for (int u = 0; u < PF; ++u) nxt[u] = *reinterpret_cast<const double2*>(Lt + 2 * min(u, NP - 1));
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int p0 = (k + 1) / 2;
    double2 cur[NP];
#pragma unroll
    for (int p = p0; p < NP; ++p)
      cur[p] = p < p0 + PF ? nxt[p - p0] : *reinterpret_cast<const double2*>(Lt + k * LD + 2 * p);
    const double dc = dn;
    if (k + 1 < N) {
      const int q0 = (k + 2) / 2;
      dn = idg[k + 1];
#pragma unroll
      for (int u = 0; u < PF; ++u)
        if (q0 + u < NP) nxt[u] = *reinterpret_cast<const double2*>(Lt + (k + 1) * LD + 2 * (q0 + u));
    }
    const double xk = x[k] * dc;
    x[k] = xk;
#pragma unroll
    for (int p = p0; 2 * p < N; ++p) {
      if (2 * p > k) x[2 * p] = fma(-cur[p].x, xk, x[2 * p]);
      if (2 * p + 1 < N) x[2 * p + 1] = fma(-cur[p].y, xk, x[2 * p + 1]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int K>
struct ElemLayout {
  using Dm = Dims<K>;
  static constexpr int D3 = Dm::D3, D2 = Dm::D2, M = Dm::M, NQD = Dm::NQD;
  static constexpr int LD = (D3 + 3) / 4 * 4;  // padded length of every D3-vector: whole 4x4 tiles
  static constexpr int PLD = LD, NQP = (NQD + 3) / 4 * 4;  // the padded basis table has rows of LD
  static constexpr int TT = LD / 4, TM = M / 4;             // tiles along D3 and along the M trace unknowns
  static constexpr int NCOL = 3 * D3 + M;                    // right-hand sides C^T | DP^T
  // W^T | Z^T; V^T = (Ls^{-1} [B | f])^T later overwrites the rows of W^T, dead by then
  static constexpr int BIG_SOLVE = NCOL * LD;
  // the basis table is staged in two halves of the points
  static constexpr int NQH = NQP / 2;
  static constexpr int BIG_STAGE = lds_stage_bytes<NQH * PLD>() / 8;
  static constexpr int BIG = BIG_SOLVE > BIG_STAGE ? BIG_SOLVE : BIG_STAGE;
  static_assert(M % 4 == 0 && NQD % 8 == 0 && NQP == NQD, "whole tiles of trace unknowns and of points");
  static_assert(M + 1 <= 3 * D3, "V^T fits in the rows of W^T");
};

template <int K>
struct CondenseSmem {
  using Ly = ElemLayout<K>;
  // half of the basis table at the points while the Gram matrices are summed, then one row
  // per solved column: W_s^T (3 D3 rows) and Z^T (M rows), then V^T = (Ls^{-1} [B | f])^T
  // (M + 1 rows) in place of W^T
  double big[Ly::BIG];
  double wkc[2 * Ly::NQD];  // (|K| w_q / kappa_q, |K| w_q c_q)
  double wf[Ly::NQD];       // |K| w_q f_q
  double Lt[Ly::LD * Ly::LD];  // M (upper tiles), then L^T
  double St[Ly::LD * Ly::LD];  // Mc, then S, then Ls^T
  double fv[Ly::LD];
  double idl[Ly::LD], ids[Ly::LD];
  double gn[4][3], gT[4], ga[9];
  int gmu[4], slot[16], fbe[4];
};

// Work item w (one element) on one workgroup of NT threads.
template <int K, int NT>
__device__ __forceinline__ void condense_element(const hdg_mesh& mesh, const Tables& tb, const double* __restrict__ kappa,
                                                 const double* __restrict__ cco, const double* __restrict__ fco,
                                                 const double* __restrict__ tau, double* __restrict__ H,
                                                 double* __restrict__ F, double* __restrict__ factors,
                                                 const int* __restrict__ elems, int nwork, double* __restrict__ Cout,
                                                 double* __restrict__ Cfout, int w) {
  using Ly = ElemLayout<K>;
  constexpr int D3 = Ly::D3, D2 = Ly::D2, M = Ly::M, NQD = Ly::NQD, LD = Ly::LD, PLD = Ly::PLD;
  constexpr int NCOL = Ly::NCOL, TT = Ly::TT, TM = Ly::TM, NW = NT / 64, NTRI = D3 * (D3 + 1) / 2;
  constexpr int NUT = TT * (TT + 1) / 2;  // upper tiles of a D3 x D3 matrix
  __shared__ __align__(16) CondenseSmem<K> sm;
  // the thread index passes through an opaque move, so the per-thread offsets and masks
  // derived from it are formed where they are used instead of being hoisted out of the
  // persistent element loop, where they would stay live across every phase
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  const int lane = t & 63, wave = t >> 6;
  // canonical tile coordinates of this lane (block blk, row tr, column tc)
  const int blk = (lane >> 2) & 3, tr = lane >> 4, tc = lane & 3;
  const int E = elems ? elems[w] : w;
  if (E < 0 || E >= mesh.nelt) return;  // uniform across the block
  double* Wt = sm.big;
  double* Zt = sm.big + 3 * D3 * LD;
  double* Vt = sm.big;  // over W^T, once B is formed
  constexpr int NQH = Ly::NQH;
  // ---- the first half of the basis table goes to LDS while the coefficients are formed
  lds_stage_wg<NQH * PLD, NW>(tb.Pt, sm.big, wave, lane);
  {
  ElemGeom g;
  load_geometry(E, mesh, tau, g);
  for (int q = t; q < NQD; q += NT) {
    const double wq = g.vol * tb.vol_w[q];
    sm.wkc[2 * q] = wq / kappa[(size_t)E * NQD + q];
    sm.wkc[2 * q + 1] = wq * cco[(size_t)E * NQD + q];
    sm.wf[q] = wq * fco[(size_t)E * NQD + q];
  }
  if (t < 16) sm.slot[t] = mesh.d_slot[16 * E + t];
  if (t < 4) {
    sm.fbe[t] = mesh.d_facebyele[4 * E + t];
    sm.gT[t] = t == 0 ? g.T[0] : t == 1 ? g.T[1] : t == 2 ? g.T[2] : g.T[3];
    sm.gmu[t] = t == 0 ? g.mu[0] : t == 1 ? g.mu[1] : t == 2 ? g.mu[2] : g.mu[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      sm.gn[t][d] = t == 0 ? g.n[0][d] : t == 1 ? g.n[1][d] : t == 2 ? g.n[2][d] : g.n[3][d];
  }
  if (t >= 64 - 9 && t < 64) {
    const int e = t - (64 - 9);
    double v = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) v = e == k ? g.a[k / 3][k % 3] : v;
    sm.ga[e] = v;
  }
  }
  lds_stage_wait();
  __syncthreads();
  // ---- right-hand-side columns C_s^T and DP_l^T (eq 5.2), fetched now and solved once L
  // is known: column c < 3 D3 is (s, i) = (c / D3, c % D3), W_s[r][i] = sum_h a[s][h]
  // Chat[h][i][r]; the others are (l, i), Z_l[r][i] = DP[mu_l][l][i][r]
  double x[D3];
  auto load_col = [&](int c) {
    if (c < 3 * D3) {
      const int s = c / D3, i = c % D3;
      const double a0 = sm.ga[3 * s], a1 = sm.ga[3 * s + 1], a2 = sm.ga[3 * s + 2];
      const double* c0 = tb.Chat + i * D3;
#pragma unroll
      for (int r = 0; r < D3; ++r) x[r] = a0 * c0[r];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < D3; ++r) x[r] = fma(a1, c0[D3 * D3 + r], x[r]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < D3; ++r) x[r] = fma(a2, c0[2 * D3 * D3 + r], x[r]);
    } else {
      const int l = (c - 3 * D3) / D2, i = (c - 3 * D3) % D2;
      const double* dp = tb.DP + ((sm.gmu[l] * 4 + l) * D2 + i) * D3;
#pragma unroll
      for (int r = 0; r < D3; ++r) x[r] = dp[r];
    }
  };
  auto store_col = [&](double* row) {
#pragma unroll
    for (int r = 0; r < LD; r += 2)
      *reinterpret_cast<double2*>(row + r) = make_double2(x[r], r + 1 < D3 ? x[r + 1 < D3 ? r + 1 : 0] : 0.0);
  };
  // ---- Gram matrices M = P^T diag(|K| w / kappa) P and Mc = P^T diag(|K| w c) P (eq 3.5,
  // eq 4.5) on the FP64 matrix cores: job j is upper tile j of both, one job per block,
  // four per wavefront instruction, four points per step; both weights come in one 16-byte
  // read and the basis operands serve both products.  The points come in two staged
  // halves; the lane of a job adds the second half's sums to the first's in LDS.  The load
  // vector f is summed beside them.
  const int fi = (NW > 1 ? NT - 65 : NT - 1) - t;  // the thread of entry fi of f
  for (int h = 0; h < 2; ++h) {
    if (h == 1) {
      __syncthreads();  // every read of the first half is done
      lds_stage_wg<NQH * PLD, NW>(tb.Pt + NQH * PLD, sm.big, wave, lane);
      lds_stage_wait();
      __syncthreads();
    }
    for (int quad = wave; quad < (NUT + 3) / 4; quad += NW) {
      const int job = min(4 * quad + blk, NUT - 1);
      int ti, tj;
      upper_pair(job, TT, ti, tj);
      const double* px = sm.big + tr * PLD + 4 * ti + tc;
      const double* py = sm.big + tr * PLD + 4 * tj + tc;
      const double* pw = sm.wkc + 2 * (h * NQH + tr);
      double am[2] = {0, 0}, ac[2] = {0, 0};  // two chains per product
#pragma unroll 6
      for (int q0 = 0; q0 < NQH; q0 += 4) {
        const int ch = (q0 / 4) & 1;
        const double2 wq = *reinterpret_cast<const double2*>(pw + 2 * q0);
        const double x = px[q0 * PLD], y = py[q0 * PLD];
        am[ch] = mfma4(x, wq.x * y, am[ch]);
        ac[ch] = mfma4(x, wq.y * y, ac[ch]);
      }
      if (4 * quad + blk < NUT) {
        const int o = (4 * ti + tr) * LD + 4 * tj + tc;
        const double vm = am[0] + am[1], vc = ac[0] + ac[1];
        sm.Lt[o] = h ? sm.Lt[o] + vm : vm;
        sm.St[o] = h ? sm.St[o] + vc : vc;
      }
    }
    if (fi >= 0 && fi < LD) {
      double sf = 0;
      if (fi < D3)
        for (int q = 0; q < NQH; ++q) sf = fma(sm.wf[h * NQH + q], sm.big[q * PLD + fi], sf);
      sm.fv[fi] = h ? sm.fv[fi] + sf : sf;
    }
  }
  __syncthreads();
  double* fa = factors ? factors + (size_t)E * (D3 * (D3 + 1) + D3) : nullptr;
  // ---- L (one wavefront); the load vector goes to the factor store
  if (wave == NW - 1) {
    const double* const parts[1] = {sm.Lt};
    wave_cholesky<D3, LD, 1>(parts, sm.Lt, sm.idl, lane);
  }
  if (fa && fi >= 0 && fi < D3) fa[D3 * (D3 + 1) + fi] = sm.fv[fi];
  __syncthreads();
  // ---- W_s = L^{-1} C_s^T, Z = L^{-1} DP^T (eq 5.2), one column per thread
  for (int c = t; c < NCOL; c += NT) {
    load_col(c);
    col_forward<D3, LD>(sm.Lt, sm.idl, x);
    store_col(sm.big + c * LD);
  }
  if (fa)
    for (int p = NT - 1 - t; p < NTRI; p += NT) {
      int i, j;
      upper_pair(p, D3, i, j);  // (i, j) with i <= j: L[j][i]
      fa[j * (j + 1) / 2 + i] = sm.Lt[i * LD + j];
    }
  __syncthreads();
  // ---- S = Mc + sum_l tau_l |e_l| PP_l + sum_s W_s^T W_s (eq 5.3), upper tiles on the
  // matrix cores (rows of W^T past D3 - 1 feed only the padding entries)
  for (int quad = wave; quad < (NUT + 3) / 4; quad += NW) {
    const int job = min(4 * quad + blk, NUT - 1);
    int ti, tj;
    upper_pair(job, TT, ti, tj);
    const int i = 4 * ti + tr, j = 4 * tj + tc, o = i * LD + j;
    double pp[4];  // the table terms are added last, so these loads overlap the products
#pragma unroll
    for (int l = 0; l < 4; ++l) pp[l] = tb.PPt[(l * PLD + i) * PLD + j];
    double acc[3] = {sm.St[o], 0, 0};  // one chain per direction
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double* px = Wt + (c * D3 + 4 * ti + tc) * LD + tr;
      const double* py = Wt + (c * D3 + 4 * tj + tc) * LD + tr;
#pragma unroll
      for (int r0 = 0; r0 < LD; r0 += 4) acc[c] = mfma4(px[r0], py[r0], acc[c]);
    }
    double sv = (acc[0] + acc[1]) + acc[2];
#pragma unroll
    for (int l = 0; l < 4; ++l) sv = fma(sm.gT[l], pp[l], sv);
    if (4 * quad + blk < NUT) sm.St[o] = sv;
  }
  __syncthreads();
  // ---- Ls (one wavefront) while the others form B_l = T_l DP_l^T + U_l^T Z_l with
  // U_l = sum_s n_{l s} W_s (eq 5.5), stored as rows of V^T
  if (wave == NW - 1) {
    const double* const parts[1] = {sm.St};
    wave_cholesky<D3, LD, 1>(parts, sm.St, sm.ids, lane);
  }
  // B^T by tiles on the matrix cores: B[i][c] = T_l DP_l[c][i] + sum_s sum_r W_s[r][i]
  // (n_{l s} Z[r][c]), l the face of column c; the normal rides on the Z operand, whose
  // element (r, tc) belongs to column 4 tcb + tc of the tile.  The tiles stay in registers
  // until every wavefront is done with W^T, whose rows then receive them.
  constexpr int NWB = NW == 1 ? 1 : NW - 1, NJ = TT * TM, NBQ = ((NJ + 3) / 4 + NWB - 1) / NWB;
  double bres[NBQ];
  if (NW == 1 || wave < NW - 1) {
#pragma unroll
    for (int u = 0; u < NBQ; ++u) {
      const int quad = wave + u * NWB;
      if (quad >= (NJ + 3) / 4) break;  // uniform across the wavefront
      const int job = min(4 * quad + blk, NJ - 1), ti = job % TT, tcb = job / TT;
      const int i = 4 * ti + tr, c = 4 * tcb + tc, l = c / D2;
      // the table term is added last, so its load overlaps the products
      const double dp = tb.DP[((sm.gmu[l] * 4 + l) * D2 + c % D2) * D3 + min(i, D3 - 1)];
      double acc[3] = {0, 0, 0};  // one chain per direction
#pragma unroll
      for (int sd = 0; sd < 3; ++sd) {
        const double ns = sm.gn[l][sd];
        const double* px = Wt + (sd * D3 + 4 * ti + tc) * LD + tr;
        const double* py = Zt + c * LD + tr;
#pragma unroll
        for (int r0 = 0; r0 < LD; r0 += 4) acc[sd] = mfma4(px[r0], ns * py[r0], acc[sd]);
      }
      bres[u] = fma(sm.gT[l], dp, (acc[0] + acc[1]) + acc[2]);
    }
  }
  __syncthreads();
  if (NW == 1 || wave < NW - 1) {
#pragma unroll
    for (int u = 0; u < NBQ; ++u) {
      const int quad = wave + u * NWB;
      if (quad >= (NJ + 3) / 4) break;
      const int job = 4 * quad + blk, ti = job % TT, tcb = job / TT;
      const int i = 4 * ti + tr, c = 4 * tcb + tc;
      if (job < NJ && i < D3) Vt[c * LD + i] = bres[u];
    }
  }
  __syncthreads();
  // ---- V = Ls^{-1} [B | f] (eq 5.6), one column per thread; the packed factor Ls
  for (int c = t; c < M + 1; c += NT) {
    const double* src = c < M ? Vt + c * LD : sm.fv;
#pragma unroll
    for (int r = 0; r < D3; ++r) x[r] = src[r];
    col_forward<D3, LD>(sm.St, sm.ids, x);
    store_col(Vt + c * LD);
  }
  if (fa)
    for (int p = NT - 1 - t; p < NTRI; p += NT) {
      int i, j;
      upper_pair(p, D3, i, j);
      fa[D3 * (D3 + 1) / 2 + j * (j + 1) / 2 + i] = sm.St[i * LD + j];
    }
  __syncthreads();
  // ---- C^K = tau DD + (n.n) Z^T Z - V^T V (upper triangle) and Cf^K = V^T (Ls^{-1} f)
  // (eq 5.6); scattered into H and F, or exported
  {
    auto emit = [&](int a, int b, double c) {
      const int la = a / D2, lb = b / D2, ia = a % D2, ib = b % D2;
      if (a == b) c += sm.gT[la];
      if (Cout) {
        Cout[((size_t)w * M + a) * M + b] = c;
        Cout[((size_t)w * M + b) * M + a] = c;
      } else {
        const size_t s1 = sm.slot[4 * la + lb];
        if (la == lb) {
          unsafeAtomicAdd(&H[(s1 * D2 + ia) * D2 + ib], c);
          if (ia != ib) unsafeAtomicAdd(&H[(s1 * D2 + ib) * D2 + ia], c);
        } else {
          const size_t s2 = sm.slot[4 * lb + la];
          H[(s1 * D2 + ia) * D2 + ib] = c;
          H[(s2 * D2 + ib) * D2 + ia] = c;
        }
      }
    };
    // job < NPT: upper tile pair (ta, tb) of C^K, the products Z^T Z and V^T V on the
    // matrix cores; NPT <= job: Cf^K for rows 4 ta .. 4 ta + 3 (the Y operand is the f
    // column of V^T for every column of the tile)
    constexpr int NPT = TM * (TM + 1) / 2, NJ = NPT + TM;
    for (int quad = wave; quad < (NJ + 3) / 4; quad += NW) {
      const int job = min(4 * quad + blk, NJ - 1);
      const bool cf = job >= NPT;
      int ta = job - NPT, tbb = 0;
      if (!cf) upper_pair(job, TM, ta, tbb);
      const double* zx = (cf ? Vt : Zt) + (4 * ta + tc) * LD + tr;
      const double* zy = (cf ? Vt + M * LD : Zt + (4 * tbb + tc) * LD) + tr;
      const double* vx = Vt + (4 * ta + tc) * LD + tr;
      const double* vy = Vt + (4 * tbb + tc) * LD + tr;
      double z2[2] = {0, 0}, v2[2] = {0, 0};  // two chains per product
#pragma unroll
      for (int r0 = 0; r0 < LD; r0 += 4) {
        z2[(r0 / 4) & 1] = mfma4(zx[r0], zy[r0], z2[(r0 / 4) & 1]);
        v2[(r0 / 4) & 1] = mfma4(vx[r0], vy[r0], v2[(r0 / 4) & 1]);
      }
      const double zz = z2[0] + z2[1], vv = v2[0] + v2[1];
      if (4 * quad + blk >= NJ) continue;
      const int a = 4 * ta + tr, b = 4 * tbb + tc;
      if (cf) {
        if (tc == 0) {
          if (Cfout)
            Cfout[(size_t)w * M + a] = zz;
          else
            unsafeAtomicAdd(&F[(size_t)sm.fbe[a / D2] * D2 + a % D2], zz);
        }
        continue;
      }
      if (a > b) continue;
      const int la = a / D2, lb = b / D2;
      const double nn = sm.gn[la][0] * sm.gn[lb][0] + sm.gn[la][1] * sm.gn[lb][1] + sm.gn[la][2] * sm.gn[lb][2];
      emit(a, b, nn * zz - vv);
    }
  }
  __syncthreads();
}

// EXPORT selects the debugging form (listed elements, C^K and Cf^K written out instead of
// scattered); the scatter form is compiled with those pointers known to be null.
template <int K, int NT, bool EXPORT>
__global__ void __launch_bounds__(NT, NT == 256 ? 2 : 1) k_condense(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                 const double* __restrict__ cco, const double* __restrict__ fco,
                                                 const double* __restrict__ tau, double* __restrict__ H,
                                                 double* __restrict__ F, double* __restrict__ factors,
                                                 const int* __restrict__ elems, int nwork, double* __restrict__ Cout,
                                                 double* __restrict__ Cfout, int xcd_remap) {
  for (int w = batch_block(xcd_remap); w < nwork; w += gridDim.x)
    condense_element<K, NT>(mesh, tb, kappa, cco, fco, tau, H, F, factors, EXPORT ? elems : nullptr, nwork,
                        EXPORT ? Cout : nullptr, EXPORT ? Cfout : nullptr, w);
}

// Degree 0, one thread per element: every block is 1 x 1, so the local solve of eq 5.1-5.6
// is scalar.  With m = M (kappa^{-1} mass), C_s the divergence entries and
// S = Mc + tauPP + sum_s C_s^2 / m, each right-hand side (b_x, b_y, b_z, b_u) gives
//   u = (b_u - sum_s C_s b_s / m) / S,   q_s = (b_s + C_s u) / m,
// with b_s = n_{l s} DP_l, b_u = -T_l DP_l for face column l and (0, 0, 0, f) for the load;
// C^K[l][m] = sum_s n_{l s} DP_l q_s^(m) + T_l DP_l u^(m) + delta_lm T_l,
// Cf^K[l] the same with the load column.  The factor store is (sqrt m, sqrt S, f), the
// layout of the per-element kernel at d3 = 1.
template <bool EXPORT>
__device__ __forceinline__ void condense_k0_element(const hdg_mesh& mesh, const Tables& tb,
                                                    const double* __restrict__ kappa, const double* __restrict__ cco,
                                                    const double* __restrict__ fco, const double* __restrict__ tau,
                                                    double* __restrict__ H, double* __restrict__ F,
                                                    double* __restrict__ factors, const int* __restrict__ elems,
                                                    double* __restrict__ Cout, double* __restrict__ Cfout, int w) {
  constexpr int NQD = 8;  // (k + 2)^3 at k = 0
  {
    const int E = EXPORT ? elems[w] : w;
    if (E < 0 || E >= mesh.nelt) return;
    ElemGeom g;
    load_geometry(E, mesh, tau, g);
    double m = 0, mc = 0, f = 0;
    for (int q = 0; q < NQD; ++q) {
      const double wq = g.vol * tb.vol_w[q], p0 = tb.P[q];
      const size_t e = (size_t)E * NQD + q;
      m += wq / kappa[e] * p0 * p0;
      mc += wq * cco[e] * p0 * p0;
      f += wq * fco[e] * p0;
    }
    double cs[3], S = mc;
    for (int l = 0; l < 4; ++l) S += g.T[l] * tb.PP[l];
    for (int sd = 0; sd < 3; ++sd) {
      cs[sd] = g.a[sd][0] * tb.Chat[0] + g.a[sd][1] * tb.Chat[1] + g.a[sd][2] * tb.Chat[2];
      S += cs[sd] * cs[sd] / m;
    }
    double dp[4], qq[5][3], uu[5];
    for (int l = 0; l < 4; ++l) dp[l] = tb.DP[g.mu[l] * 4 + l];
    for (int c = 0; c < 5; ++c) {  // columns: faces 0..3, then the load
      double bs[3], bu;
      if (c < 4) {
        for (int sd = 0; sd < 3; ++sd) bs[sd] = g.n[c][sd] * dp[c];
        bu = -g.T[c] * dp[c];
      } else {
        bs[0] = bs[1] = bs[2] = 0.0;
        bu = f;
      }
      double r = bu;
      for (int sd = 0; sd < 3; ++sd) r -= cs[sd] * bs[sd] / m;
      uu[c] = r / S;
      for (int sd = 0; sd < 3; ++sd) qq[c][sd] = (bs[sd] + cs[sd] * uu[c]) / m;
    }
    // the upper triangle of C^K (c >= l), mirrored, so that H is exactly symmetric; column 4
    // is the load, reached for every l
    for (int l = 0; l < 4; ++l) {
      const double a0 = g.n[l][0] * dp[l], a1 = g.n[l][1] * dp[l], a2 = g.n[l][2] * dp[l], a3 = g.T[l] * dp[l];
      for (int c = l; c < 5; ++c) {
        double v = a0 * qq[c][0] + a1 * qq[c][1] + a2 * qq[c][2] + a3 * uu[c];
        if (c == 4) {
          if (EXPORT)
            Cfout[(size_t)w * 4 + l] = v;
          else
            unsafeAtomicAdd(&F[mesh.d_facebyele[4 * E + l]], v);
          continue;
        }
        if (c == l) v += g.T[l];
        if (EXPORT) {
          Cout[((size_t)w * 4 + l) * 4 + c] = v;
          Cout[((size_t)w * 4 + c) * 4 + l] = v;
        } else if (c == l) {
          unsafeAtomicAdd(&H[mesh.d_slot[16 * E + 5 * l]], v);
        } else {
          H[mesh.d_slot[16 * E + 4 * l + c]] = v;
          H[mesh.d_slot[16 * E + 4 * c + l]] = v;
        }
      }
    }
    if (!EXPORT && factors) {
      double* fa = factors + (size_t)E * 3;
      fa[0] = sqrt(m);
      fa[1] = sqrt(S);
      fa[2] = f;
    }
  }
}

template <bool EXPORT>
__global__ void __launch_bounds__(256) k_condense_k0(hdg_mesh mesh, Tables tb, const double* __restrict__ kappa,
                                                     const double* __restrict__ cco, const double* __restrict__ fco,
                                                     const double* __restrict__ tau, double* __restrict__ H,
                                                     double* __restrict__ F, double* __restrict__ factors,
                                                     const int* __restrict__ elems, int nwork,
                                                     double* __restrict__ Cout, double* __restrict__ Cfout) {
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < nwork; w += gridDim.x * blockDim.x)
    condense_k0_element<EXPORT>(mesh, tb, kappa, cco, fco, tau, H, F, factors, elems, Cout, Cfout, w);
}

// Batched degree 0: thread u takes element u - unit_begin of its mesh (same arithmetic, so the
// same bits as a separate call).
__global__ void __launch_bounds__(256) k_batch_condense_k0(const BatchItem* __restrict__ items, int nitems,
                                                           int total_units, Tables tb) {
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < total_units; u += gridDim.x * blockDim.x) {
    const BatchItem* it = items + batch_find(items, nitems, u);
    condense_k0_element<false>(as_global(it->mesh), tb, as_global(it->kappa), as_global(it->c), as_global(it->f),
                               as_global(it->tau), as_global(it->H), as_global(it->F), as_global(it->factors),
                               nullptr, nullptr, nullptr, u - it->unit_begin);
  }
}

// Persistent batched form: work unit u is element u - unit_begin of its mesh.
template <int K, int NT>
__global__ void __launch_bounds__(NT, NT == 256 ? 2 : 1) k_batch_condense(const BatchItem* __restrict__ items, int nitems, int total_units,
                                                       Tables tb, int xcd_remap) {
  for (int u = batch_block(xcd_remap); u < total_units; u += gridDim.x) {
    const BatchItem* it = items + batch_find(items, nitems, u);
    condense_element<K, NT>(as_global(it->mesh), tb, as_global(it->kappa), as_global(it->c), as_global(it->f),
                            as_global(it->tau), as_global(it->H), as_global(it->F), as_global(it->factors), nullptr,
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
  const hdg_mesh& m = *mesh;
  const Tables& tb = disc->dev;
  if constexpr (K == 0) {  // scalar local systems: one thread per element
    const unsigned g0 = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65535));
    if (Cout)
      k_condense_k0<true><<<g0, 256, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout);
    else {
      timer_begin("k_condense", s);
      k_condense_k0<false><<<g0, 256, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, nullptr, (int)n, nullptr,
                                              nullptr);
      timer_end("k_condense", s);
    }
    HDG_CHECK_LAUNCH("k_condense_k0");
    return HDG_OK;
  } else {
  const hdg_tile_config lc = launch_config(K);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)lc.workgroups_per_cu * device_cu_count()));
  const int rm = lc.xcd_remap;
  if (Cout) {  // export form: one shape is enough
    k_condense<K, 256, true><<<grid, 256, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout, rm);
  } else {
    timer_begin("k_condense", s);
    switch (lc.waves_per_element) {
      case 1: k_condense<K, 64, false><<<grid, 64, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout, rm); break;
      case 2: k_condense<K, 128, false><<<grid, 128, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout, rm); break;
      case 4: k_condense<K, 256, false><<<grid, 256, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout, rm); break;
      default: k_condense<K, 512, false><<<grid, 512, 0, s>>>(m, tb, kappa, c, f, tau, H, F, factors, elems, (int)n, Cout, Cfout, rm); break;
    }
    timer_end("k_condense", s);
  }
  HDG_CHECK_LAUNCH("k_condense");
  return HDG_OK;
  }
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
                             double* dws = nullptr, size_t ws_bytes = 0) {
  if (disc->host.k >= 5)
    return dispatch_condense_big(disc, mesh, kappa, c, f, tau, H, F, factors, elems, n, Cout, Cfout, dws, ws_bytes, s);
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
    case 0:  // one thread per element; the workgroup shape of the other degrees does not apply
      k_batch_condense_k0<<<(unsigned)std::max(1, std::min((total_units + 255) / 256, 65535)), 256, 0, s>>>(
          d_items, nitems, total_units, tb);
      HDG_CHECK_LAUNCH("k_batch_condense_k0");
      return HDG_OK;
    case 4: return launch_batch_element<4>(tb, d_items, nitems, total_units, grid, xcd_remap, waves, s);
  }
  return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "batched condensation: unsupported degree");
}

// ---- the one singular configuration of the method (Section 1: the system has a unique
// solution when kappa > 0, c >= 0 and tau_K is not identically zero on any K, unless there is
// no Dirichlet face and c vanishes everywhere: then every constant trace with u = const,
// q = 0 solves the homogeneous system).  The flag is a file-scope device variable, so the
// check allocates nothing; it is cleared by a kernel, not a memset.
__device__ int g_reaction_positive;

__global__ void k_flag_clear() { g_reaction_positive = 0; }

__global__ void k_any_positive(const double* __restrict__ c, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (c[i] > 0.0) g_reaction_positive = 1;  // every writer stores the same value
}

hdg_status check_not_singular(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_c, hipStream_t s,
                              const char* who) {
  if (mesh->ndir > 0) return HDG_OK;
  const int64_t n = mesh->nelt * (int64_t)disc->host.nqd;
  k_flag_clear<<<1, 1, 0, s>>>();
  k_any_positive<<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, s>>>(d_c, n);
  HDG_CHECK_LAUNCH("k_any_positive");
  int flag = 0;
  hipError_t e = hipMemcpyFromSymbolAsync(&flag, HIP_SYMBOL(g_reaction_positive), sizeof(int), 0,
                                          hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return check_hip(e, who);
  if (!flag)
    return set_error(HDG_ERR_SINGULAR, std::string(who) +
                                           ": no Dirichlet face and c == 0 at every point: constants span the kernel");
  return HDG_OK;
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
  st = check_not_singular(disc, mesh, d_c, (hipStream_t)stream, "hdg_assemble_condense");
  if (st) return st;
  return dispatch_condense(disc, mesh, d_kappa, d_c, d_f, d_tau, d_H, d_F, d_factors, nullptr, mesh->nelt, nullptr,
                           nullptr, (hipStream_t)stream);
}

extern "C" hdg_status hdg_condense_workspace_size(const hdg_disc* disc, const hdg_mesh* mesh, size_t* bytes) {
  if (!disc || !mesh || !bytes) return set_error(HDG_ERR_INVALID_ARG, "hdg_condense_workspace_size: NULL argument");
  const int k = disc->host.k;
  *bytes = (k >= 1 && k <= 3) ? condense_ws_bytes(disc->host.d2, mesh->nelt)
           : k >= 5           ? condense_big_workspace_bytes(k, mesh->nelt)
                              : 0;
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
  st = check_not_singular(disc, mesh, d_c, (hipStream_t)stream, "hdg_assemble_condense_ws");
  if (st) return st;
  return dispatch_condense(disc, mesh, d_kappa, d_c, d_f, d_tau, d_H, d_F, d_factors, nullptr, mesh->nelt, nullptr,
                           nullptr, (hipStream_t)stream, need ? (double*)d_ws : nullptr, ws_bytes);
}

namespace hdg {
hdg_status condense_static_workspace(size_t need, double** ws);
size_t condense_scratch_capacity();
}  // namespace hdg

extern "C" hdg_status hdg_condense_noalloc_capacity(size_t* bytes) {
  if (!bytes) return set_error(HDG_ERR_INVALID_ARG, "hdg_condense_noalloc_capacity: NULL argument");
  *bytes = condense_scratch_capacity();
  return HDG_OK;
}

extern "C" hdg_status hdg_assemble_condense_noalloc(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                                    const double* d_c, const double* d_f, const double* d_tau,
                                                    double* d_H, double* d_F, double* d_factors, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_assemble_condense_noalloc");
  if (st) return st;
  if (!d_kappa || !d_c || !d_f || !d_tau || !d_H || !d_F || !mesh->d_face_elem)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_assemble_condense_noalloc: NULL array");
  size_t need = 0;
  hdg_condense_workspace_size(disc, mesh, &need);
  double* ws = nullptr;
  st = condense_static_workspace(need, &ws);
  if (st) return st;
  st = check_not_singular(disc, mesh, d_c, (hipStream_t)stream, "hdg_assemble_condense_noalloc");
  if (st) return st;
  return dispatch_condense(disc, mesh, d_kappa, d_c, d_f, d_tau, d_H, d_F, d_factors, nullptr, mesh->nelt, nullptr,
                           nullptr, (hipStream_t)stream, ws, need);
}

namespace hdg {
hdg_status dispatch_condense_tile_bdm(const hdg_disc* disc, const hdg_mesh* mesh, const double* kappa, const double* c,
                                      const double* f, double* H, double* F, double* factors, double* dws,
                                      hipStream_t s);
}  // namespace hdg

extern "C" hdg_status hdg_assemble_condense_bdm(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                                const double* d_c, const double* d_f, double* d_H, double* d_F,
                                                double* d_factors, void* d_ws, size_t ws_bytes, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_assemble_condense_bdm");
  if (st) return st;
  if (disc->host.k < 1 || disc->host.k > 3)
    return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_assemble_condense_bdm: degrees 1..3");
  if (!d_kappa || !d_c || !d_f || !d_H || !d_F || !d_factors || !mesh->d_face_elem)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_assemble_condense_bdm: NULL array");
  size_t need = 0;
  hdg_condense_workspace_size(disc, mesh, &need);
  if (!d_ws || ws_bytes < need) return set_error(HDG_ERR_WORKSPACE, "hdg_assemble_condense_bdm: workspace too small");
  st = check_not_singular(disc, mesh, d_c, (hipStream_t)stream, "hdg_assemble_condense_bdm");
  if (st) return st;
  return dispatch_condense_tile_bdm(disc, mesh, d_kappa, d_c, d_f, d_H, d_F, d_factors, (double*)d_ws,
                                    (hipStream_t)stream);
}

extern "C" hdg_status hdg_export_local(const hdg_disc* disc, const hdg_mesh* mesh, const double* d_kappa,
                                       const double* d_c, const double* d_f, const double* d_tau,
                                       const int32_t* d_elems, int64_t n, double* d_C, double* d_Cf, void* stream) {
  hdg_status st = check_disc_mesh(disc, mesh, "hdg_export_local");
  if (st) return st;
  if (!d_kappa || !d_c || !d_f || !d_tau || !d_elems || !d_C || !d_Cf || n < 0)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_export_local: NULL array");
  if (disc->host.k > kMaxBatchDegree)
    return set_error(HDG_ERR_UNSUPPORTED_DEGREE, "hdg_export_local: degrees 0..4");
  return dispatch_condense(disc, mesh, d_kappa, d_c, d_f, d_tau, nullptr, nullptr, nullptr, d_elems, n, d_C, d_Cf,
                           (hipStream_t)stream);
}
