// Reference-element tables for degree k (Sections 3-4 of the paper), built on the host
// in long double: Stroud conical-product Gauss-Jacobi rules (eq 3.1 and the face rule of
// Section 4), the orthonormal hierarchical Dubiner bases on the reference tetrahedron and
// triangle (eq 3.3, Section 4) with their reference gradients, and the element-independent
// matrices C^# (eq 3.7), PP_l (eq 4.5), DP_{mu,l} (eq 4.10) and the P_{k+1} stiffness
// tables of the postprocess (eq 9.11).
//
// Conventions (shared with the rest of the library):
//   * rules: n points per collapsed direction with Jacobi weights (1-a)^0, (1-b)^1,
//     (1-c)^2 (triangle: (1-a)^0, (1-b)^1); a varies slowest; weights scaled to sum 1;
//   * bases: on xi = 2 x - 1, psi_pqr = P_p(a) ((1-b)/2)^p P_q^{(2p+1,0)}(b)
//     ((1-c)/2)^{p+q} P_r^{(2p+2q+2,0)}(c) scaled by sqrt((2p+1)(2p+2q+2)(2p+2q+2r+3)/6)
//     and psi_pq = P_p(a) ((1-b)/2)^p P_q^{(2p+1,0)}(b) scaled by sqrt((2p+1)(p+q+1)),
//     ordered by total degree, then p, then q.  They are evaluated in homogenised form,
//     Y^p P_p(X/Y) etc., which gives analytic gradients away from the collapsed vertex.
#include <cmath>
#include <stdexcept>

#include "hdg_internal.h"

namespace hdg {
namespace {

using ld = long double;

// Jacobi polynomial P_n^{(a,b)}(x) and its derivative, three-term recurrence.
void jacobi(int n, ld a, ld b, ld x, ld* val, ld* der) {
  auto eval = [&](int nn, ld aa, ld bb) -> ld {
    if (nn < 0) return 0;
    ld p0 = 1;
    if (nn == 0) return p0;
    ld p1 = ((aa + bb + 2) * x + (aa - bb)) / 2;
    for (int j = 2; j <= nn; ++j) {
      ld c1 = 2 * j * (j + aa + bb) * (2 * j + aa + bb - 2);
      ld c2 = (2 * j + aa + bb - 1) * ((2 * j + aa + bb) * (2 * j + aa + bb - 2) * x + aa * aa - bb * bb);
      ld c3 = 2 * (j + aa - 1) * (j + bb - 1) * (2 * j + aa + bb);
      ld p2 = (c2 * p1 - c3 * p0) / c1;
      p0 = p1;
      p1 = p2;
    }
    return p1;
  };
  *val = eval(n, a, b);
  *der = n == 0 ? 0 : (n + a + b + 1) / 2 * eval(n - 1, a + 1, b + 1);
}

// Gauss-Jacobi nodes for the weight (1-x)^a on [-1,1] by Newton's method with deflation;
// weights proportional to 1 / ((1 - x^2) P_n'(x)^2).
void gauss_jacobi(int n, ld a, std::vector<ld>& x, std::vector<ld>& w) {
  x.assign(n, 0);
  w.assign(n, 0);
  const ld pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < n; ++i) {
    ld r = -std::cos((2 * i + 1) * pi / (2 * n));
    if (i > 0) r = (r + x[i - 1]) / 2;
    for (int it = 0; it < 200; ++it) {
      ld v, d;
      jacobi(n, a, 0, r, &v, &d);
      ld s = 0;
      for (int j = 0; j < i; ++j) s += 1 / (r - x[j]);
      ld delta = -v / (d - s * v);
      r += delta;
      if (std::fabs(delta) < 1e-30L) break;
    }
    x[i] = r;
  }
  for (int i = 0; i < n; ++i) {
    ld v, d;
    jacobi(n, a, 0, x[i], &v, &d);
    w[i] = 1 / ((1 - x[i] * x[i]) * d * d);
  }
}

// Y^p P_p^{(al,0)}(X/Y) and its partial derivatives in X and Y.
void homog(int p, ld al, ld X, ld Y, ld* F, ld* FX, ld* FY) {
  if (p == 0) {
    *F = 1;
    *FX = 0;
    *FY = 0;
    return;
  }
  ld a = X / Y, v, d;
  jacobi(p, al, 0, a, &v, &d);
  ld yp1 = std::pow(Y, (ld)(p - 1));
  *F = yp1 * Y * v;
  *FX = yp1 * d;
  *FY = yp1 * (p * v - a * d);
}

// 3-D orthonormal Dubiner basis of degree <= k at reference point x (3), with gradients.
void dubiner3(int k, const ld* x, std::vector<ld>& val, std::vector<ld>* grad /*[3][d3]*/) {
  const int d3 = dim3(k);
  val.assign(d3, 0);
  if (grad) grad->assign(3 * d3, 0);
  ld x1 = 2 * x[0] - 1, x2 = 2 * x[1] - 1, x3 = 2 * x[2] - 1;
  ld X = 2 + 2 * x1 + x2 + x3, Y = -x2 - x3, U = 1 + 2 * x2 + x3, V = 1 - x3;
  // d(X,Y,U,V)/d(xi1,xi2,xi3)
  const ld dX[3] = {2, 1, 1}, dY[3] = {0, -1, -1}, dU[3] = {0, 2, 1}, dV[3] = {0, 0, -1};
  int idx = 0;
  for (int n = 0; n <= k; ++n)
    for (int p = 0; p <= n; ++p)
      for (int q = 0; q <= n - p; ++q, ++idx) {
        int r = n - p - q;
        ld F, FX, FY, G, GU, GV, H, Hd;
        homog(p, 0, X, Y, &F, &FX, &FY);
        homog(q, 2 * p + 1, U, V, &G, &GU, &GV);
        jacobi(r, 2 * p + 2 * q + 2, 0, x3, &H, &Hd);
        ld scale = std::sqrt((ld)(2 * p + 1) * (2 * p + 2 * q + 2) * (2 * p + 2 * q + 2 * r + 3) / 6) /
                   std::pow((ld)2, (ld)(p + q));
        val[idx] = F * G * H * scale;
        if (grad) {
          for (int i = 0; i < 3; ++i) {
            ld dF = FX * dX[i] + FY * dY[i];
            ld dG = GU * dU[i] + GV * dV[i];
            ld dH = i == 2 ? Hd : 0;
            // d/dx_i = 2 d/dxi_i
            (*grad)[i * d3 + idx] = 2 * scale * (dF * G * H + F * dG * H + F * G * dH);
          }
        }
      }
}

// 2-D orthonormal Dubiner basis of degree <= k at reference point (s, t).
void dubiner2(int k, ld s, ld t, std::vector<ld>& val) {
  val.assign(dim2(k), 0);
  ld x1 = 2 * s - 1, x2 = 2 * t - 1;
  ld X = 1 + 2 * x1 + x2, Y = 1 - x2;
  int idx = 0;
  for (int n = 0; n <= k; ++n)
    for (int p = 0; p <= n; ++p, ++idx) {
      int q = n - p;
      ld F, FX, FY, G, Gd;
      homog(p, 0, X, Y, &F, &FX, &FY);
      jacobi(q, 2 * p + 1, 0, x2, &G, &Gd);
      val[idx] = F * G * std::sqrt((ld)(2 * p + 1) * (p + q + 1)) / std::pow((ld)2, (ld)p);
    }
}

}  // namespace

HostTables build_tables(int k, int nq) {
  HostTables t;
  t.k = k;
  t.nq = nq;
  t.d3 = dim3(k);
  t.d2 = dim2(k);
  t.d3p = dim3(k + 1);
  t.nqd = nq * nq * nq;
  t.nqd2 = nq * nq;
  const int d3 = t.d3, d2 = t.d2, d3p = t.d3p, nqd = t.nqd, nqd2 = t.nqd2;

  // ---- rules
  std::vector<ld> a, wa, b, wb, c, wc;
  gauss_jacobi(nq, 0, a, wa);
  gauss_jacobi(nq, 1, b, wb);
  gauss_jacobi(nq, 2, c, wc);
  std::vector<ld> vp(3 * nqd), vw(nqd), tp(2 * nqd2), tw(nqd2);
  ld sw = 0;
  for (int i = 0, q = 0; i < nq; ++i)
    for (int j = 0; j < nq; ++j)
      for (int l = 0; l < nq; ++l, ++q) {
        ld xi1 = (1 + a[i]) * (1 - b[j]) * (1 - c[l]) / 4 - 1;
        ld xi2 = (1 + b[j]) * (1 - c[l]) / 2 - 1;
        ld xi3 = c[l];
        vp[3 * q] = (xi1 + 1) / 2;
        vp[3 * q + 1] = (xi2 + 1) / 2;
        vp[3 * q + 2] = (xi3 + 1) / 2;
        vw[q] = wa[i] * wb[j] * wc[l];
        sw += vw[q];
      }
  for (auto& w : vw) w /= sw;
  ld st = 0;
  for (int i = 0, r = 0; i < nq; ++i)
    for (int j = 0; j < nq; ++j, ++r) {
      ld xi1 = (1 + a[i]) * (1 - b[j]) / 2 - 1, xi2 = b[j];
      tp[2 * r] = (xi1 + 1) / 2;
      tp[2 * r + 1] = (xi2 + 1) / 2;
      tw[r] = wa[i] * wb[j];
      st += tw[r];
    }
  for (auto& w : tw) w /= st;

  // ---- basis values
  std::vector<ld> P(nqd * d3), Pg(3 * nqd * d3), P1g(3 * nqd * d3p), val, grad;
  for (int q = 0; q < nqd; ++q) {
    dubiner3(k, &vp[3 * q], val, &grad);
    for (int j = 0; j < d3; ++j) {
      P[q * d3 + j] = val[j];
      for (int i = 0; i < 3; ++i) Pg[(i * nqd + q) * d3 + j] = grad[i * d3 + j];
    }
    dubiner3(k + 1, &vp[3 * q], val, &grad);
    for (int j = 0; j < d3p; ++j)
      for (int i = 0; i < 3; ++i) P1g[(i * nqd + q) * d3p + j] = grad[i * d3p + j];
  }
  std::vector<ld> D(nqd2 * d2), Pface(4 * nqd2 * d3), Dmu(6 * nqd2 * d2);
  for (int r = 0; r < nqd2; ++r) {
    ld s = tp[2 * r], tt = tp[2 * r + 1];
    dubiner2(k, s, tt, val);
    for (int i = 0; i < d2; ++i) D[r * d2 + i] = val[i];
    // eq 2.5: points of the four faces of the reference tetrahedron
    const ld fpts[4][3] = {{s, tt, 0}, {s, 0, tt}, {0, s, tt}, {s, tt, 1 - s - tt}};
    for (int l = 0; l < 4; ++l) {
      dubiner3(k, fpts[l], val, nullptr);
      for (int j = 0; j < d3; ++j) Pface[(l * nqd2 + r) * d3 + j] = val[j];
    }
    // eq 2.2: F_mu(s, t)
    const ld fm[6][2] = {{s, tt}, {tt, s}, {tt, 1 - s - tt}, {s, 1 - s - tt}, {1 - s - tt, s}, {1 - s - tt, tt}};
    for (int mu = 0; mu < 6; ++mu) {
      dubiner2(k, fm[mu][0], fm[mu][1], val);
      for (int i = 0; i < d2; ++i) Dmu[(mu * nqd2 + r) * d2 + i] = val[i];
    }
  }

  // ---- reference matrices
  std::vector<ld> Chat(3 * d3 * d3, 0), PP(4 * d3 * d3, 0), DP(24 * d2 * d3, 0), Shat(6 * d3p * d3p, 0);
  for (int h = 0; h < 3; ++h)
    for (int i = 0; i < d3; ++i)
      for (int j = 0; j < d3; ++j) {
        ld s = 0;
        for (int q = 0; q < nqd; ++q) s += vw[q] * P[q * d3 + i] * Pg[(h * nqd + q) * d3 + j];
        Chat[(h * d3 + i) * d3 + j] = s / 6;
      }
  for (int l = 0; l < 4; ++l)
    for (int i = 0; i < d3; ++i)
      for (int j = 0; j < d3; ++j) {
        ld s = 0;
        for (int r = 0; r < nqd2; ++r) s += tw[r] * Pface[(l * nqd2 + r) * d3 + i] * Pface[(l * nqd2 + r) * d3 + j];
        PP[(l * d3 + i) * d3 + j] = s;
      }
  for (int mu = 0; mu < 6; ++mu)
    for (int l = 0; l < 4; ++l)
      for (int i = 0; i < d2; ++i)
        for (int j = 0; j < d3; ++j) {
          ld s = 0;
          for (int r = 0; r < nqd2; ++r) s += tw[r] * Dmu[(mu * nqd2 + r) * d2 + i] * Pface[(l * nqd2 + r) * d3 + j];
          DP[(((mu * 4) + l) * d2 + i) * d3 + j] = s;
        }
  // Inverse of the last d2 columns of each DP_{mu,l}: the face moments of the degree-k modes
  // that are orthogonal to P_{k-1}(K).  A polynomial of P_k(K) orthogonal to P_{k-1}(K) that
  // vanishes on a face is zero, so this d2 x d2 block is invertible (HDG projection, eq 9.13).
  // Gauss-Jordan with partial pivoting in long double.
  std::vector<ld> DPtopinv(24 * d2 * d2, 0);
  for (int ml = 0; ml < 24; ++ml) {
    std::vector<ld> a(d2 * 2 * d2, 0);
    for (int i = 0; i < d2; ++i) {
      for (int j = 0; j < d2; ++j) a[i * 2 * d2 + j] = DP[(ml * d2 + i) * d3 + (d3 - d2) + j];
      a[i * 2 * d2 + d2 + i] = 1;
    }
    for (int c = 0; c < d2; ++c) {
      int piv = c;
      for (int r = c + 1; r < d2; ++r)
        if (std::fabs(a[r * 2 * d2 + c]) > std::fabs(a[piv * 2 * d2 + c])) piv = r;
      if (std::fabs(a[piv * 2 * d2 + c]) < 1e-12L) throw std::runtime_error("singular top-mode face block");
      if (piv != c)
        for (int j = 0; j < 2 * d2; ++j) std::swap(a[c * 2 * d2 + j], a[piv * 2 * d2 + j]);
      const ld inv = 1 / a[c * 2 * d2 + c];
      for (int j = 0; j < 2 * d2; ++j) a[c * 2 * d2 + j] *= inv;
      for (int r = 0; r < d2; ++r)
        if (r != c) {
          const ld f = a[r * 2 * d2 + c];
          if (f != 0)
            for (int j = 0; j < 2 * d2; ++j) a[r * 2 * d2 + j] -= f * a[c * 2 * d2 + j];
        }
    }
    for (int i = 0; i < d2; ++i)
      for (int j = 0; j < d2; ++j) DPtopinv[(ml * d2 + i) * d2 + j] = a[i * 2 * d2 + d2 + j];
  }
  const int pairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  for (int pidx = 0; pidx < 6; ++pidx) {
    int h = pairs[pidx][0], g = pairs[pidx][1];
    for (int i = 0; i < d3p; ++i)
      for (int j = 0; j < d3p; ++j) {
        ld s = 0;
        for (int q = 0; q < nqd; ++q) {
          ld v = P1g[(h * nqd + q) * d3p + i] * P1g[(g * nqd + q) * d3p + j];
          if (h != g) v += P1g[(g * nqd + q) * d3p + i] * P1g[(h * nqd + q) * d3p + j];
          s += vw[q] * v;
        }
        Shat[(pidx * d3p + i) * d3p + j] = s / 6;
      }
  }

  // ---- pack
  TableOffsets& o = t.off;
  int pos = 0;
  auto take = [&](int n) {
    int p = pos;
    pos += (n + 7) & ~7;  // 64-byte alignment of every table
    return p;
  };
  o.vol_pts = take(3 * nqd);
  o.vol_w = take(nqd);
  o.lambda = take(4 * nqd);
  o.P = take(nqd * d3);
  o.Pg = take(3 * nqd * d3);
  o.tri_pts = take(2 * nqd2);
  o.tri_w = take(nqd2);
  o.xi = take(3 * nqd2);
  o.D = take(nqd2 * d2);
  o.Pface = take(4 * nqd2 * d3);
  o.Chat = take(3 * d3 * d3);
  o.PP = take(4 * d3 * d3);
  o.DP = take(24 * d2 * d3);
  o.P1g = take(3 * nqd * d3p);
  o.Shat = take(6 * d3p * d3p);
  o.DPtopinv = take(24 * d2 * d2);
  o.Dmu = take(6 * nqd2 * d2);
  const int D3P4 = (d3 + 3) / 4 * 4, D2P4 = (d2 + 3) / 4 * 4, NQP = (nqd + 3) / 4 * 4;
  t.d3p4 = D3P4;
  t.d2p4 = D2P4;
  t.nqp = NQP;
  o.Pt = take(NQP * D3P4);
  o.ChatT = take(3 * D3P4 * D3P4);
  o.PPt = take(4 * D3P4 * D3P4);
  o.DPT = take(24 * D3P4 * D2P4);
  const int D3PP4 = (d3p + 3) / 4 * 4, TS = D3PP4 / 4, NUS = TS * (TS + 1) / 2;
  t.d3pp4 = D3PP4;
  o.P1gt = take(3 * NQP * D3PP4);
  o.Shatt = take(6 * NUS * 16);
  o.total = pos;
  t.data.assign(pos, 0.0);
  auto put = [&](int off, const std::vector<ld>& v) {
    for (size_t i = 0; i < v.size(); ++i) t.data[off + i] = (double)v[i];
  };
  put(o.vol_pts, vp);
  put(o.vol_w, vw);
  std::vector<ld> lam(4 * nqd);
  for (int q = 0; q < nqd; ++q) {
    lam[4 * q] = 1 - vp[3 * q] - vp[3 * q + 1] - vp[3 * q + 2];
    for (int i = 0; i < 3; ++i) lam[4 * q + 1 + i] = vp[3 * q + i];
  }
  put(o.lambda, lam);
  put(o.P, P);
  put(o.Pg, Pg);
  put(o.tri_pts, tp);
  put(o.tri_w, tw);
  std::vector<ld> xi(3 * nqd2);
  for (int r = 0; r < nqd2; ++r) {
    xi[3 * r] = 1 - tp[2 * r] - tp[2 * r + 1];
    xi[3 * r + 1] = tp[2 * r];
    xi[3 * r + 2] = tp[2 * r + 1];
  }
  put(o.xi, xi);
  put(o.D, D);
  put(o.Pface, Pface);
  put(o.Chat, Chat);
  put(o.PP, PP);
  put(o.DP, DP);
  put(o.P1g, P1g);
  put(o.Shat, Shat);
  put(o.DPtopinv, DPtopinv);
  put(o.Dmu, Dmu);
  for (int q = 0; q < nqd; ++q)
    for (int j = 0; j < d3; ++j) t.data[o.Pt + q * D3P4 + j] = (double)P[q * d3 + j];
  for (int h = 0; h < 3; ++h)
    for (int i = 0; i < d3; ++i)
      for (int j = 0; j < d3; ++j) t.data[o.ChatT + (h * D3P4 + i) * D3P4 + j] = (double)Chat[(h * d3 + j) * d3 + i];
  for (int l = 0; l < 4; ++l)
    for (int i = 0; i < d3; ++i)
      for (int j = 0; j < d3; ++j) t.data[o.PPt + (l * D3P4 + i) * D3P4 + j] = (double)PP[(l * d3 + i) * d3 + j];
  for (int ml = 0; ml < 24; ++ml)
    for (int i = 0; i < d3; ++i)
      for (int j = 0; j < d2; ++j) t.data[o.DPT + (ml * D3P4 + i) * D2P4 + j] = (double)DP[(ml * d2 + j) * d3 + i];
  for (int h = 0; h < 3; ++h)
    for (int q = 0; q < nqd; ++q)
      for (int i = 0; i < d3p; ++i)
        t.data[o.P1gt + (h * NQP + q) * D3PP4 + i] = (double)P1g[(h * nqd + q) * d3p + i];
  for (int p = 0; p < 6; ++p)
    for (int I = 0; I < TS; ++I)
      for (int N = I; N < TS; ++N) {
        const int u = I * TS - I * (I - 1) / 2 + (N - I);
        for (int r = 0; r < 4; ++r)
          for (int c = 0; c < 4; ++c) {
            const int i = 4 * I + r, j = 4 * N + c;
            if (i < d3p && j < d3p)
              t.data[o.Shatt + (p * NUS + u) * 16 + 4 * r + c] = (double)Shat[(p * d3p + i) * d3p + j];
          }
      }
  return t;
}

}  // namespace hdg
