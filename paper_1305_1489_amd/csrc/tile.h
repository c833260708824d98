// 4x4-tile dense linear algebra on the FP64 matrix cores of gfx950 (v_mfma_f64_4x4x4f64).
//
// The instruction runs four independent 4x4x4 products per wavefront, one per group of 16
// lanes ("block").  Lane l belongs to block (l >> 2) & 3 and, inside a tile, to row
// r = l >> 4 and column c = l & 3.  With every operand stored in this layout ("canonical
// tile": the lane holds X[r][c]), the instruction computes
//     D = X^T Y + C
// for the two 4x4 source tiles X, Y and the accumulator C.  Each block carries one
// element, so a wavefront works on four elements at once and every per-element matrix is
// an array of tiles, one double per lane per tile.
//
// A product A B of tiled matrices therefore needs the tiles of A^T (A "in transposed
// storage") and B in normal storage; Gram products X^T Y need both in normal storage.
#pragma once

#include "device_common.h"

namespace hdg {

__device__ __forceinline__ double mfma4(double x, double y, double acc) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(x, y, acc, 0, 0, 0);
}

// Index of tile (I, N), I <= N, in the packed upper triangle of a T x T tile matrix.
__host__ __device__ constexpr int utile(int I, int N, int T) { return I * T - I * (I - 1) / 2 + (N - I); }

// Ordering of LDS traffic inside one wavefront (the wavefront runs in lockstep; the fences
// keep the compiler from moving LDS accesses across this point).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The copy's LDS writes arrive through the vector-memory return path, not the LDS queue of
// the wavefront, so nothing orders them after LDS reads and writes that the wavefront issued
// earlier and that are still in flight; the compiler inserts no wait for that hazard (a
// wavefront-scope fence emits none, and it may leave loads of the destination outstanding
// when it schedules their consumers later).  Every copy therefore first drains the
// wavefront's LDS traffic, so that a buffer read just before it (the Gram weights before
// the divergence tables land in the same space) is read before it is overwritten.
__device__ __forceinline__ void lds_drain() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Asynchronous copy of an element-independent table (N doubles, N even, 16-byte aligned)
// from global memory straight into LDS, 1 KB per wavefront instruction and no registers:
// lane t of copy i moves doubles 128 i + 2t, +1 (clamped to the table, so the source is
// never overrun); the LDS destination must hold whole kilobytes, ceil(8N / 1024) of them.
// Completion is awaited with lds_stage_wait() before the first read.
template <int N>
__device__ __forceinline__ void lds_stage(const double* __restrict__ src, double* dst, int lane) {
  static_assert(N % 2 == 0, "tables are staged in pairs of doubles");
  constexpr int NI = (N * 8 + 1023) / 1024;
  lds_drain();
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int o = min(128 * i + 2 * lane, N - 2);
    __builtin_amdgcn_global_load_lds(src + o, (__attribute__((address_space(3))) void*)(dst + 128 * i), 16, 0, 0);
  }
}
template <int N>
constexpr int lds_stage_bytes() { return (N * 8 + 1023) / 1024 * 1024; }
// The same copy shared by the NW wavefronts of a workgroup (wavefront w issues copies
// w, w + NW, ...); every wavefront awaits its own copies with lds_stage_wait() and the
// workgroup then synchronises.  The other wavefronts' reads of the destination must be
// ordered before the copy by a workgroup barrier, as for any LDS write.
template <int N, int NW>
__device__ __forceinline__ void lds_stage_wg(const double* __restrict__ src, double* dst, int wave, int lane) {
  static_assert(N % 2 == 0, "tables are staged in pairs of doubles");
  constexpr int NI = (N * 8 + 1023) / 1024;
  lds_drain();
  for (int i = wave; i < NI; i += NW) {
    const int o = min(128 * i + 2 * lane, N - 2);
    __builtin_amdgcn_global_load_lds(src + o, (__attribute__((address_space(3))) void*)(dst + 128 * i), 16, 0, 0);
  }
}
__device__ __forceinline__ void lds_stage_wait() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  wave_lds_sync();
}

// 1/sqrt(s) for a positive normal s (a Cholesky pivot): the hardware estimate (relative
// error about 2^-23) refined by two Newton steps y <- y (3/2 - s y^2 / 2), to round-off.
__device__ __forceinline__ double pivot_rsqrt(double s) {
  double y = __builtin_amdgcn_rsq(s);
  const double hs = 0.5 * s;
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-hs * y, y, 0.5), y);
  return y;
}

// Upper Cholesky of one 4x4 SPD tile per block (A = U^T U) and the inverse V = U^{-1}.
// Every lane of the block reads the whole tile through LDS and factors it redundantly;
// it returns its own entries U[r][c] and V[r][c].  xch: 64 doubles of LDS, private to the
// wavefront when WAVE (then only the wavefront is synchronised), else to the workgroup.
template <bool WAVE = false>
__device__ __forceinline__ void diag_chol4(double a_rc, double* xch, double& u_rc, double& v_rc) {
  const int lane = threadIdx.x & 63, r = lane >> 4, c = lane & 3, blk = (lane >> 2) & 3;
  if (WAVE) wave_lds_sync(); else __syncthreads();
  xch[blk * 16 + r * 4 + c] = a_rc;
  if (WAVE) wave_lds_sync(); else __syncthreads();
  double a[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) a[i][j] = xch[blk * 16 + i * 4 + j];
  // one reciprocal square root per pivot and no division: FP64 vector work is issued on
  // the matrix cores' time, and this chain is serial
  double u[4][4] = {}, v[4][4] = {}, dinv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double s = a[i][i];
#pragma unroll
    for (int k = 0; k < i; ++k) s -= u[k][i] * u[k][i];
    dinv[i] = pivot_rsqrt(s);
    u[i][i] = s * dinv[i];
#pragma unroll
    for (int j = i + 1; j < 4; ++j) {
      double t = a[i][j];
#pragma unroll
      for (int k = 0; k < i; ++k) t -= u[k][i] * u[k][j];
      u[i][j] = t * dinv[i];
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v[j][j] = dinv[j];
#pragma unroll
    for (int i = j - 1; i >= 0; --i) {
      double t = 0;
#pragma unroll
      for (int k = i + 1; k <= j; ++k) t += u[i][k] * v[k][j];
      v[i][j] = -t * dinv[i];
    }
  }
  double ur = 0, vr = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (i == r && j == c) {
        ur = u[i][j];
        vr = v[i][j];
      }
  u_rc = ur;
  v_rc = vr;
}

// The value v of lane src (cross-lane permute, no LDS storage).
__device__ __forceinline__ double lane_read(double v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Transpose of each block's 4x4 tile: the lane (r, c) receives X[c][r].
__device__ __forceinline__ double tile_transpose(double v) {
  const int lane = threadIdx.x & 63;
  return lane_read(v, 16 * (lane & 3) + (lane & 12) + (lane >> 4));
}

// Inverse of the upper Cholesky factor: given U (packed upper tiles) and Vd[J] =
// U(J,J)^{-1}, returns Ui = U^{-1} as packed upper tiles.  Computed as L^{-1} = U^{-T} by
// block forward substitution on the identity (natural operand forms for the matrix
// cores), then each tile transposed into place.
template <int T>
__device__ __forceinline__ void tile_upper_inverse(const double (&U)[T * (T + 1) / 2], const double (&Vd)[T],
                                                   double (&Ui)[T * (T + 1) / 2]) {
  const int lane = threadIdx.x & 63;
  const double eye = ((lane >> 4) == (lane & 3)) ? 1.0 : 0.0;
#pragma unroll
  for (int J = 0; J < T; ++J) {
    double X[T];
#pragma unroll
    for (int I = J; I < T; ++I) {
      double acc = 0.0;
#pragma unroll
      for (int K = J; K < I; ++K) acc = mfma4(U[utile(K, I, T)], X[K], acc);
      X[I] = mfma4(Vd[I], (I == J ? eye : 0.0) - acc, 0.0);  // X = L^{-1}(:, J)
    }
#pragma unroll
    for (int I = J; I < T; ++I) Ui[utile(J, I, T)] = tile_transpose(X[I]);  // U^{-1}(J,I) = L^{-1}(I,J)^T
  }
}

// Blocked upper Cholesky in place on the packed upper tiles A (T x T tiles, symmetric
// matrix): afterwards A holds U (A = U^T U) and Vd[J] = U(J,J)^{-1}.
template <int T, bool WAVE = false>
__device__ __forceinline__ void tile_cholesky(double (&A)[T * (T + 1) / 2], double (&Vd)[T], double* xch) {
#pragma unroll
  for (int J = 0; J < T; ++J) {
    double u, v;
    diag_chol4<WAVE>(A[utile(J, J, T)], xch, u, v);
    A[utile(J, J, T)] = u;
    Vd[J] = v;
    // panel: U(J,I) = U(J,J)^{-T} A(J,I)
#pragma unroll
    for (int I = J + 1; I < T; ++I) A[utile(J, I, T)] = mfma4(v, A[utile(J, I, T)], 0.0);
    // trailing update: A(I',I) -= U(J,I')^T U(J,I)
#pragma unroll
    for (int Ip = J + 1; Ip < T; ++Ip)
#pragma unroll
      for (int I = Ip; I < T; ++I) A[utile(Ip, I, T)] -= mfma4(A[utile(J, Ip, T)], A[utile(J, I, T)], 0.0);
  }
}

// Value of lane l (uniform) of v, for the whole wavefront.
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __hiloint2double(hi, lo);
}

// Cholesky factor (eq 5.1, eq 5.4) of the N x N SPD matrix whose upper triangle is
// A[0] + ... + A[NP-1] (row-major, leading dimension LD; entry (i, k) kept at
// [min(i, k)][max(i, k)]), by one wavefront: lane i holds row i in registers; pass j
// broadcasts column j lane by lane (v_readlane), updates the trailing rows with it while
// still unscaled and then scales it; column j + 1 is updated first, so the next pivot's
// reciprocal square root overlaps the rest of the pass.
// Writes L^T to Lt (Lt[k][i] = L[i][k] for k <= i) and the reciprocal diagonal to idg.
// Lt may alias A[0]: every lane has read its row before any lane writes.
template <int N, int LD, int NP>
__device__ __forceinline__ void wave_cholesky(const double* const (&A)[NP], double* Lt, double* idg, int lane) {
  const int i = min(lane, N - 1);
  double a[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int o = k < i ? k * LD + i : i * LD + k;
    double s = A[0][o];
#pragma unroll
    for (int p = 1; p < NP; ++p) s += A[p][o];
    a[k] = s;
    if (k % 8 == 7) __builtin_amdgcn_sched_barrier(0);
  }
  double myid = 0;
  double piv = lane_bcast(a[0], 0), id = pivot_rsqrt(piv);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double t = a[j] * (id * id);
    double pn = 1.0, idn = 1.0;
    if (j + 1 < N) {  // column j + 1 first, so the next pivot's square root overlaps this pass
      a[j + 1] = fma(-t, lane_bcast(a[j], j + 1), a[j + 1]);
      pn = lane_bcast(a[j + 1], j + 1);
      idn = pivot_rsqrt(pn);
    }
#pragma unroll
    for (int k = j + 2; k < N; ++k) {
      a[k] = fma(-t, lane_bcast(a[j], k), a[k]);
      if ((k - j) % 8 == 0) __builtin_amdgcn_sched_barrier(0);  // bounds the broadcasts in flight
    }
    a[j] = lane == j ? piv * id : a[j] * id;
    if (lane == j) myid = id;
    piv = pn;
    id = idn;
    __builtin_amdgcn_sched_barrier(0);
  }
  if (lane < N) {
#pragma unroll
    for (int k = 0; k < N; ++k)
      if (k <= lane) Lt[k * LD + lane] = a[k];
    idg[lane] = myid;
  }
}

}  // namespace hdg
