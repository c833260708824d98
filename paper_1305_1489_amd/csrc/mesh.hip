// Mesh expansion on the device (Section 2, "Data structure", expanded form).
//
// Faces are found by sorting the 4 Nelt sorted-vertex-triple keys of the element faces
// (eq 2.1 order) with a stable least-significant-digit radix sort that carries the
// element-face index 4K+l, followed by a segmented unique.  Every integer output is a
// deterministic function of the input: faces are numbered by ascending key, the two
// holders of an interior face appear in ascending 4K+l order, and the block pattern of
// the trace matrix is sorted by column.
#include <algorithm>
#include <cstdio>

#include "hdg_internal.h"

namespace hdg {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;                      // items per thread in the radix passes
constexpr int kTile = kThreads * kItems;       // items per block
constexpr int kDigitBits = 4;
constexpr int kBuckets = 1 << kDigitBits;

__device__ inline void raise_error(int* err, int code) { atomicCAS(err, 0, code); }

__device__ inline void sort3(int& a, int& b, int& c) {
  if (a > b) { int t = a; a = b; b = t; }
  if (b > c) { int t = b; b = c; c = t; }
  if (a > b) { int t = a; a = b; b = t; }
}

__device__ inline unsigned long long face_key(int a, int b, int c, int bl) {
  sort3(a, b, c);
  return ((unsigned long long)a << (2 * bl)) | ((unsigned long long)b << bl) | (unsigned long long)c;
}

// eq 2.1 local faces
__constant__ int c_local[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {3, 1, 2}};
// eq 2.2: images of (w1, w2, w3) under F_mu
__constant__ int c_fmu[6][3] = {{1, 2, 3}, {1, 3, 2}, {3, 1, 2}, {3, 2, 1}, {2, 3, 1}, {2, 1, 3}};

// ---- keys, volumes, outward normals, orientation check
__global__ void k_face_keys(const double* __restrict__ X, const int* __restrict__ T, int nelt, int nver, int bl,
                            unsigned long long* __restrict__ keys, int* __restrict__ vals, double* __restrict__ vol,
                            double* __restrict__ normals, int* err) {
  int K = blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= nelt) return;
  int v[4];
  double p[4][3];
  for (int i = 0; i < 4; ++i) {
    v[i] = T[4 * K + i];
    if (v[i] < 0 || v[i] >= nver) {
      raise_error(err, HDG_ERR_INVALID_ARG);
      v[i] = 0;
    }
    for (int d = 0; d < 3; ++d) p[i][d] = X[3 * v[i] + d];
  }
  double e1[3], e2[3], e3[3];
  for (int d = 0; d < 3; ++d) {
    e1[d] = p[1][d] - p[0][d];
    e2[d] = p[2][d] - p[0][d];
    e3[d] = p[3][d] - p[0][d];
  }
  double det = (e1[1] * e2[2] - e1[2] * e2[1]) * e3[0] + (e1[2] * e2[0] - e1[0] * e2[2]) * e3[1] +
               (e1[0] * e2[1] - e1[1] * e2[0]) * e3[2];
  if (!(det > 0)) raise_error(err, HDG_ERR_MESH_ORIENTATION);
  vol[K] = det / 6.0;
  for (int l = 0; l < 4; ++l) {
    int a = c_local[l][0], b = c_local[l][1], c = c_local[l][2];
    double u[3], w[3];
    for (int d = 0; d < 3; ++d) {
      u[d] = p[b][d] - p[a][d];
      w[d] = p[c][d] - p[a][d];
    }
    // faces 1 and 3 of eq 2.1 point inwards: flip them
    double s = (l == 0 || l == 2) ? -0.5 : 0.5;
    normals[12 * K + 3 * l + 0] = s * (u[1] * w[2] - u[2] * w[1]);
    normals[12 * K + 3 * l + 1] = s * (u[2] * w[0] - u[0] * w[2]);
    normals[12 * K + 3 * l + 2] = s * (u[0] * w[1] - u[1] * w[0]);
    keys[4 * K + l] = face_key(v[a], v[b], v[c], bl);
    vals[4 * K + l] = 4 * K + l;
  }
}

// ---- stable LSD radix sort, 4-bit digits
__global__ void k_radix_count(const unsigned long long* __restrict__ keys, int n, int shift, int nb,
                              int* __restrict__ hist) {
  __shared__ int cnt[kBuckets];
  if (threadIdx.x < kBuckets) cnt[threadIdx.x] = 0;
  __syncthreads();
  int base = blockIdx.x * kTile + threadIdx.x * kItems;
  int loc[kBuckets];
  for (int d = 0; d < kBuckets; ++d) loc[d] = 0;
  for (int j = 0; j < kItems; ++j) {
    int i = base + j;
    if (i < n) loc[(keys[i] >> shift) & (kBuckets - 1)]++;
  }
  for (int d = 0; d < kBuckets; ++d)
    if (loc[d]) atomicAdd(&cnt[d], loc[d]);
  __syncthreads();
  if (threadIdx.x < kBuckets) hist[threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void k_radix_scatter(const unsigned long long* __restrict__ kin, const int* __restrict__ vin,
                                unsigned long long* __restrict__ kout, int* __restrict__ vout, int n, int shift,
                                int nb, const int* __restrict__ offs) {
  __shared__ int pre[kBuckets][kThreads];
  int base = blockIdx.x * kTile + threadIdx.x * kItems;
  int loc[kBuckets];
  for (int d = 0; d < kBuckets; ++d) loc[d] = 0;
  for (int j = 0; j < kItems; ++j) {
    int i = base + j;
    if (i < n) loc[(kin[i] >> shift) & (kBuckets - 1)]++;
  }
  for (int d = 0; d < kBuckets; ++d) pre[d][threadIdx.x] = loc[d];
  __syncthreads();
  if (threadIdx.x < kBuckets) {  // exclusive prefix over threads, one digit per thread
    int run = 0;
    for (int t = 0; t < kThreads; ++t) {
      int c = pre[threadIdx.x][t];
      pre[threadIdx.x][t] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int d = 0; d < kBuckets; ++d) loc[d] = offs[d * nb + blockIdx.x] + pre[d][threadIdx.x];
  for (int j = 0; j < kItems; ++j) {
    int i = base + j;
    if (i < n) {
      unsigned long long k = kin[i];
      int d = (k >> shift) & (kBuckets - 1);
      int o = loc[d]++;
      kout[o] = k;
      vout[o] = vin[i];
    }
  }
}

// ---- exclusive scan of int32 (three kernels), out[n] = total
constexpr int kScanTile = 1024;  // 256 threads x 4

__device__ int block_exclusive_scan(int v, int* sh, int* total) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kThreads; o <<= 1) {
    int x = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  int incl = sh[t];
  *total = sh[kThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_local(const int* in, int* out, int n, int* __restrict__ sums) {
  __shared__ int sh[kThreads];
  int base = blockIdx.x * kScanTile + threadIdx.x * 4;
  int v[4], s = 0;
  for (int j = 0; j < 4; ++j) {
    v[j] = base + j < n ? in[base + j] : 0;
    s += v[j];
  }
  int tot;
  int ex = block_exclusive_scan(s, sh, &tot);
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) out[base + j] = ex;
    ex += v[j];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_scan_sums(int* __restrict__ sums, int nb, int* __restrict__ total_out) {
  __shared__ int sh[kThreads];
  int carry = 0;
  for (int base = 0; base < nb; base += kThreads) {
    int i = base + threadIdx.x;
    int v = i < nb ? sums[i] : 0;
    int tot;
    int ex = block_exclusive_scan(v, sh, &tot);
    if (i < nb) sums[i] = ex + carry;
    carry += tot;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_add(int* __restrict__ out, int n, const int* __restrict__ sums) {
  int i = blockIdx.x * kScanTile + threadIdx.x;
  int add = sums[blockIdx.x];
  for (int j = 0; j < 4; ++j, i += kThreads)
    if (i < n) out[i] += add;
}

// ---- segments
__global__ void k_seg_flags(const unsigned long long* __restrict__ keys, int n, int* __restrict__ flag, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
  if (i >= 2 && keys[i] == keys[i - 2]) raise_error(err, HDG_ERR_MESH_NONCONFORMING);
}

__global__ void k_segments(const unsigned long long* __restrict__ keys, const int* __restrict__ vals,
                           const int* __restrict__ flag, const int* __restrict__ start_of, int n, int nfc,
                           const int* __restrict__ T, unsigned long long* __restrict__ ukeys,
                           int* __restrict__ faces, int* __restrict__ ftype, int* __restrict__ face_elem,
                           int* __restrict__ facebyele, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int f = start_of[i] + flag[i] - 1;  // exclusive scan + own flag = face number
  if (f < 0 || f >= nfc) {
    raise_error(err, HDG_ERR_BOUNDARY_UNLISTED);
    return;
  }
  int v = vals[i];
  facebyele[v] = f;
  if (flag[i]) {
    ukeys[f] = keys[i];
    int K = v >> 2, l = v & 3;
    faces[3 * f + 0] = T[4 * K + c_local[l][0]];
    faces[3 * f + 1] = T[4 * K + c_local[l][1]];
    faces[3 * f + 2] = T[4 * K + c_local[l][2]];
    ftype[f] = 0;
    face_elem[2 * f] = v;
    face_elem[2 * f + 1] = (i + 1 < n && keys[i + 1] == keys[i]) ? vals[i + 1] : -1;
  }
}

// ---- boundary lists
__global__ void k_boundary_rows(const int* __restrict__ rows, int nrows, int code, const double* __restrict__ X,
                                int nver, int bl, const unsigned long long* __restrict__ ukeys, int nfc,
                                const int* __restrict__ face_elem, const double* __restrict__ normals,
                                int* __restrict__ faces, int* __restrict__ ftype, int* __restrict__ out_list,
                                int* err) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int a = rows[3 * r], b = rows[3 * r + 1], c = rows[3 * r + 2];
  if (a < 0 || b < 0 || c < 0 || a >= nver || b >= nver || c >= nver || a == b || b == c || a == c) {
    raise_error(err, HDG_ERR_BOUNDARY_INVALID);
    return;
  }
  unsigned long long key = face_key(a, b, c, bl);
  int lo = 0, hi = nfc - 1, f = -1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    unsigned long long km = ukeys[mid];
    if (km == key) { f = mid; break; }
    if (km < key) lo = mid + 1; else hi = mid - 1;
  }
  if (f < 0 || face_elem[2 * f + 1] >= 0) {
    raise_error(err, HDG_ERR_BOUNDARY_INVALID);
    return;
  }
  if (atomicCAS(&ftype[f], 0, code) != 0) {
    raise_error(err, HDG_ERR_BOUNDARY_INVALID);
    return;
  }
  // the listed orientation must agree with the holder's outward normal
  double u[3], w[3];
  for (int d = 0; d < 3; ++d) {
    u[d] = X[3 * b + d] - X[3 * a + d];
    w[d] = X[3 * c + d] - X[3 * a + d];
  }
  double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
  int v = face_elem[2 * f];
  const double* no = normals + 12 * (v >> 2) + 3 * (v & 3);
  if (!(n[0] * no[0] + n[1] * no[1] + n[2] * no[2] > 0)) raise_error(err, HDG_ERR_MESH_ORIENTATION);
  faces[3 * f + 0] = a;
  faces[3 * f + 1] = b;
  faces[3 * f + 2] = c;
  out_list[r] = f;
}

__global__ void k_unlisted(const int* __restrict__ face_elem, const int* __restrict__ ftype, int nfc, int* err) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfc) return;
  if (face_elem[2 * f + 1] < 0 && ftype[f] == 0) raise_error(err, HDG_ERR_BOUNDARY_UNLISTED);
}

__global__ void k_perm_area(const double* __restrict__ X, const int* __restrict__ T, const int* __restrict__ faces,
                            const int* __restrict__ facebyele, int nelt, int nfc, int* __restrict__ perm,
                            double* __restrict__ area, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 4 * nelt) {
    int K = i >> 2, l = i & 3;
    int f = facebyele[i];
    int L0 = T[4 * K + c_local[l][0]], L1 = T[4 * K + c_local[l][1]], L2 = T[4 * K + c_local[l][2]];
    int G[3] = {faces[3 * f], faces[3 * f + 1], faces[3 * f + 2]};
    int mu = 0;
    for (int m = 0; m < 6; ++m)
      if (L0 == G[c_fmu[m][0] - 1] && L1 == G[c_fmu[m][1] - 1] && L2 == G[c_fmu[m][2] - 1]) mu = m + 1;
    if (mu == 0) raise_error(err, HDG_ERR_MESH_NONCONFORMING);
    perm[i] = mu;
  }
  if (i < nfc) {
    const int* g = faces + 3 * i;
    double u[3], w[3];
    for (int d = 0; d < 3; ++d) {
      u[d] = X[3 * g[1] + d] - X[3 * g[0] + d];
      w[d] = X[3 * g[2] + d] - X[3 * g[0] + d];
    }
    double n0 = u[1] * w[2] - u[2] * w[1], n1 = u[2] * w[0] - u[0] * w[2], n2 = u[0] * w[1] - u[1] * w[0];
    area[i] = 0.5 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  }
}

// ---- block pattern of H
__global__ void k_row_counts(const int* __restrict__ face_elem, int nfc, int* __restrict__ cnt) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < nfc) cnt[f] = face_elem[2 * f + 1] >= 0 ? 7 : 4;
  if (f == nfc) cnt[f] = 0;
}

__global__ void k_bsr_cols(const int* __restrict__ face_elem, const int* __restrict__ facebyele,
                           const int* __restrict__ row_ptr, int nfc, int* __restrict__ col_idx,
                           int* __restrict__ diag) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfc) return;
  int cols[7], n = 0;
  cols[n++] = f;
  for (int s = 0; s < 2; ++s) {
    int v = face_elem[2 * f + s];
    if (v < 0) continue;
    int K = v >> 2, l = v & 3;
    for (int m = 0; m < 4; ++m)
      if (m != l) cols[n++] = facebyele[4 * K + m];
  }
  for (int i = 1; i < n; ++i) {  // insertion sort
    int x = cols[i], j = i - 1;
    while (j >= 0 && cols[j] > x) { cols[j + 1] = cols[j]; --j; }
    cols[j + 1] = x;
  }
  int base = row_ptr[f];
  for (int i = 0; i < n; ++i) {
    col_idx[base + i] = cols[i];
    if (cols[i] == f) diag[f] = base + i;
  }
}

__global__ void k_slots(const int* __restrict__ facebyele, const int* __restrict__ row_ptr,
                        const int* __restrict__ col_idx, int nelt, int* __restrict__ slot, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 16 * nelt) return;
  int K = i >> 4, l = (i >> 2) & 3, m = i & 3;
  int f = facebyele[4 * K + l], g = facebyele[4 * K + m];
  int s = -1;
  for (int p = row_ptr[f]; p < row_ptr[f + 1]; ++p)
    if (col_idx[p] == g) s = p;
  if (s < 0) raise_error(err, HDG_ERR_MESH_NONCONFORMING);
  slot[i] = s;
}

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

struct Carve {
  char* p;
  size_t left;
  bool ok = true;
  template <class T>
  T* take(size_t n) {
    size_t bytes = (n * sizeof(T) + 255) & ~size_t(255);
    if (bytes > left) {
      ok = false;
      return nullptr;
    }
    T* r = reinterpret_cast<T*>(p);
    p += bytes;
    left -= bytes;
    return r;
  }
};

size_t scan_scratch_ints(long long n) { return (size_t)cdiv(n, kScanTile) + 1; }

hdg_status launch_scan(const int* in, int* out, long long n, int* sums, int* total, hipStream_t s) {
  int nb = std::max(1, cdiv(n, kScanTile));
  k_scan_local<<<nb, kThreads, 0, s>>>(in, out, (int)n, sums);
  k_scan_sums<<<1, kThreads, 0, s>>>(sums, nb, total);
  k_scan_add<<<nb, kThreads, 0, s>>>(out, (int)n, sums);
  HDG_CHECK_LAUNCH("scan");
  return HDG_OK;
}

int bitlen(long long v) {
  int b = 0;
  while (v > 0) { ++b; v >>= 1; }
  return std::max(b, 1);
}

}  // namespace
}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_mesh_sizes(hdg_mesh* mesh, size_t* ws_bytes) {
  if (!mesh || !ws_bytes) return set_error(HDG_ERR_INVALID_ARG, "hdg_mesh_sizes: NULL argument");
  if (mesh->nver < 4 || mesh->nelt < 1 || mesh->ndir < 0 || mesh->nneu < 0)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_mesh_sizes: invalid sizes");
  if (mesh->nver > (1 << 21)) return set_error(HDG_ERR_INVALID_ARG, "hdg_mesh_sizes: more than 2^21 vertices");
  long long nbd = mesh->ndir + mesh->nneu;
  if ((4 * mesh->nelt + nbd) % 2) return set_error(HDG_ERR_INVALID_ARG, "hdg_mesh_sizes: 4 nelt + nbd is odd");
  if (4 * mesh->nelt > (1LL << 30)) return set_error(HDG_ERR_INVALID_ARG, "hdg_mesh_sizes: mesh too large");
  mesh->nfc = (4 * mesh->nelt + nbd) / 2;
  mesh->nnzb = mesh->nfc + 12 * mesh->nelt;
  long long n = 4 * mesh->nelt;
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  add(n * sizeof(unsigned long long));                   // keys (double buffer)
  add(n * sizeof(unsigned long long));
  add(n * sizeof(int));                                  // vals (double buffer)
  add(n * sizeof(int));
  add((size_t)kBuckets * cdiv(n, kTile) * sizeof(int));  // histogram / offsets
  add(n * sizeof(int));                                  // flags
  add(n * sizeof(int));                                  // scan output
  add(scan_scratch_ints(std::max<long long>(n, kBuckets * cdiv(n, kTile))) * sizeof(int));
  add(mesh->nfc * sizeof(unsigned long long));           // unique keys
  add((mesh->nfc + 1) * sizeof(int));                    // row counts
  add(4 * sizeof(int));                                  // error flag, totals
  *ws_bytes = b;
  return HDG_OK;
}

extern "C" hdg_status hdg_mesh_expand(hdg_mesh* mesh, void* d_ws, size_t ws_bytes, void* stream) {
  size_t need = 0;
  hdg_status st = hdg_mesh_sizes(mesh, &need);
  if (st) return st;
  if (!d_ws || ws_bytes < need) return set_error(HDG_ERR_WORKSPACE, "hdg_mesh_expand: workspace too small");
  if (!mesh->d_coords || !mesh->d_elements || (mesh->ndir && !mesh->d_dirichlet) || (mesh->nneu && !mesh->d_neumann) ||
      !mesh->d_faces || !mesh->d_ftype || (mesh->ndir && !mesh->d_dirfaces) || (mesh->nneu && !mesh->d_neufaces) ||
      !mesh->d_facebyele || !mesh->d_perm || !mesh->d_volume || !mesh->d_area || !mesh->d_normals ||
      !mesh->d_face_elem || !mesh->d_row_ptr || !mesh->d_col_idx || !mesh->d_diag || !mesh->d_slot)
    return set_error(HDG_ERR_INVALID_ARG, "hdg_mesh_expand: NULL array");
  hipStream_t s = (hipStream_t)stream;
  const long long n = 4 * mesh->nelt;
  const int nelt = (int)mesh->nelt, nfc = (int)mesh->nfc;
  const int nb = cdiv(n, kTile);
  Carve cv{(char*)d_ws, ws_bytes};
  auto* keys0 = cv.take<unsigned long long>(n);
  auto* keys1 = cv.take<unsigned long long>(n);
  auto* vals0 = cv.take<int>(n);
  auto* vals1 = cv.take<int>(n);
  auto* hist = cv.take<int>((size_t)kBuckets * nb);
  auto* flag = cv.take<int>(n);
  auto* scan = cv.take<int>(n);
  auto* sums = cv.take<int>(scan_scratch_ints(std::max<long long>(n, (long long)kBuckets * nb)));
  auto* ukeys = cv.take<unsigned long long>(nfc);
  auto* rowcnt = cv.take<int>(nfc + 1);
  auto* misc = cv.take<int>(4);  // [0] error flag, [1] total of the last scan
  if (!cv.ok) return set_error(HDG_ERR_WORKSPACE, "hdg_mesh_expand: workspace carve failed");
  const int T256 = 256;
  hipError_t e = hipMemsetAsync(misc, 0, 4 * sizeof(int), s);
  if (e != hipSuccess) return check_hip(e, "hdg_mesh_expand: memset");
  const int bl = bitlen(mesh->nver - 1);
  k_face_keys<<<cdiv(nelt, T256), T256, 0, s>>>(mesh->d_coords, mesh->d_elements, nelt, (int)mesh->nver, bl, keys0,
                                                 vals0, mesh->d_volume, mesh->d_normals, misc);
  HDG_CHECK_LAUNCH("k_face_keys");
  // radix sort of the keys (3 bl significant bits)
  unsigned long long *kin = keys0, *kout = keys1;
  int *vin = vals0, *vout = vals1;
  for (int shift = 0; shift < 3 * bl; shift += kDigitBits) {
    k_radix_count<<<nb, kThreads, 0, s>>>(kin, (int)n, shift, nb, hist);
    if ((st = launch_scan(hist, hist, (long long)kBuckets * nb, sums, misc + 1, s))) return st;
    k_radix_scatter<<<nb, kThreads, 0, s>>>(kin, vin, kout, vout, (int)n, shift, nb, hist);
    HDG_CHECK_LAUNCH("radix");
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  k_seg_flags<<<cdiv(n, T256), T256, 0, s>>>(kin, (int)n, flag, misc);
  if ((st = launch_scan(flag, scan, n, sums, misc + 1, s))) return st;
  // number of distinct faces must equal the size implied by the boundary lists
  int hbuf[2] = {0, 0};
  e = hipMemcpyAsync(hbuf, misc, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return check_hip(e, "hdg_mesh_expand: readback");
  if (hbuf[0]) return set_error(hbuf[0], "hdg_mesh_expand: invalid mesh (element orientation, vertex ids or a face in more than two elements)");
  if (hbuf[1] > nfc) return set_error(HDG_ERR_BOUNDARY_UNLISTED, "hdg_mesh_expand: boundary faces missing from the Dirichlet/Neumann lists");
  if (hbuf[1] < nfc) return set_error(HDG_ERR_BOUNDARY_INVALID, "hdg_mesh_expand: boundary lists hold triangles that are not boundary faces");
  k_segments<<<cdiv(n, T256), T256, 0, s>>>(kin, vin, flag, scan, (int)n, nfc, mesh->d_elements, ukeys, mesh->d_faces,
                                            mesh->d_ftype, mesh->d_face_elem, mesh->d_facebyele, misc);
  if (mesh->ndir)
    k_boundary_rows<<<cdiv(mesh->ndir, T256), T256, 0, s>>>(mesh->d_dirichlet, (int)mesh->ndir, 1, mesh->d_coords,
                                                            (int)mesh->nver, bl, ukeys, nfc, mesh->d_face_elem,
                                                            mesh->d_normals, mesh->d_faces, mesh->d_ftype,
                                                            mesh->d_dirfaces, misc);
  if (mesh->nneu)
    k_boundary_rows<<<cdiv(mesh->nneu, T256), T256, 0, s>>>(mesh->d_neumann, (int)mesh->nneu, 2, mesh->d_coords,
                                                            (int)mesh->nver, bl, ukeys, nfc, mesh->d_face_elem,
                                                            mesh->d_normals, mesh->d_faces, mesh->d_ftype,
                                                            mesh->d_neufaces, misc);
  k_unlisted<<<cdiv(nfc, T256), T256, 0, s>>>(mesh->d_face_elem, mesh->d_ftype, nfc, misc);
  k_perm_area<<<cdiv(std::max<long long>(n, nfc), T256), T256, 0, s>>>(mesh->d_coords, mesh->d_elements, mesh->d_faces,
                                                                      mesh->d_facebyele, nelt, nfc, mesh->d_perm,
                                                                      mesh->d_area, misc);
  k_row_counts<<<cdiv(nfc + 1, T256), T256, 0, s>>>(mesh->d_face_elem, nfc, rowcnt);
  HDG_CHECK_LAUNCH("expand");
  if ((st = launch_scan(rowcnt, mesh->d_row_ptr, nfc + 1, sums, misc + 1, s))) return st;
  k_bsr_cols<<<cdiv(nfc, T256), T256, 0, s>>>(mesh->d_face_elem, mesh->d_facebyele, mesh->d_row_ptr, nfc,
                                              mesh->d_col_idx, mesh->d_diag);
  k_slots<<<cdiv(16LL * nelt, T256), T256, 0, s>>>(mesh->d_facebyele, mesh->d_row_ptr, mesh->d_col_idx, nelt,
                                                   mesh->d_slot, misc);
  HDG_CHECK_LAUNCH("pattern");
  e = hipMemcpyAsync(hbuf, misc, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return check_hip(e, "hdg_mesh_expand: readback");
  if (hbuf[0]) return set_error(hbuf[0], "hdg_mesh_expand: invalid boundary lists or mesh");
  if (hbuf[1] != mesh->nnzb) return set_error(HDG_ERR_MESH_NONCONFORMING, "hdg_mesh_expand: block count mismatch");
  return HDG_OK;
}
