// SVD of the bordered middle matrix of the incremental SVD (Sec. 4.2,
// Eq. (middleMat), (svdMiddleMat)):
//
//     Q = [ diag(s)  l ]      s_0 >= s_1 >= ... >= s_{r-1} > 0,  p >= 0.
//         [    0     p ]
//
// Q Q^T = diag(d)^2 + z z^T with d = (s, 0) and z = (l, p), so the singular
// values are the roots of the secular equation
//     f(sigma) = 1 + sum_j z_j^2 / (d_j^2 - sigma^2) = 0,
// one in each gap of the d's (plus one above d_0), and the singular vectors
// have closed forms
//     u_t ~ z_t / (d_t^2 - sigma^2),   v_t ~ d_t z_t / (d_t^2 - sigma^2) (t < r),  v_r ~ -1
// (v = Q^T u / sigma and the secular equation give the last entry).  This is
// the divide-and-conquer SVD update (Bunch-Nielsen-Sorensen; Gu and
// Eisenstat, "A divide-and-conquer algorithm for the bidiagonal SVD", 1995):
//   * deflation: a coordinate with |z_t| <= tol is decoupled (sigma = d_t,
//     unit vectors); two coordinates whose d's differ by <= tol are rotated
//     so that one z vanishes;
//   * each root is stored as sigma = d_o + tau with o the nearer end of its
//     gap, so sigma - d_t = (d_o - d_t) + tau keeps its relative accuracy;
//     tau is found by Newton's method safeguarded by bisection;
//   * z is recomputed from the computed roots (Loewner's formula) so that
//     the vectors are orthogonal to working precision.
// The p coordinate (d = 0) is never rotated; when it deflates the snapshot
// is dependent on the basis and its zero singular value is dropped, as the
// algorithm does for p below its tolerance.
//
// Every routine is written for one thread and takes plain arrays, so the
// kernel can spread the per-root and per-vector work over threads while a
// host build runs the same code in loops.
#pragma once

#include <math.h>
#include <stdint.h>

#ifdef __HIPCC__
#define BSVD_FN __host__ __device__ inline
#else
#define BSVD_FN inline
#endif

namespace bsvd {

constexpr double kEps = 2.220446049250313e-16;  // machine epsilon of double
constexpr int kMaxNewton = 200;

// Work arrays of one problem of n = r + 1 coordinates (r = rank before the
// update).  The caller owns the storage (LDS in the kernel).
struct Problem {
  int r;           // coordinates 0..r-1 carry (s, l), coordinate r carries (0, p)
  double* d;       // [n] d_t
  double* z;       // [n] z_t, rotated and deflated in place
  int* act;        // [n] active coordinates in order (descending d), count na
  int na;
  int* rot_i;      // [r] rotation pairs (kept, deflated), count nrot
  int* rot_j;
  double* rot_c;
  double* rot_s;
  int nrot;
  bool p_active;   // the p coordinate is active (the snapshot is not dependent)
};

// Deflation (sequential).  d, z filled by the caller; `dependent` forces the
// p coordinate out.  Returns the tolerance used.
BSVD_FN double deflate(Problem& P, bool dependent) {
  const int r = P.r;
  double zz = 0.0;
  for (int t = 0; t <= r; ++t) zz += P.z[t] * P.z[t];
  const double dmax = r > 0 ? P.d[0] : 0.0;
  const double tol = 8.0 * kEps * fmax(dmax, sqrt(zz));
  if (dependent || fabs(P.z[r]) <= tol) P.z[r] = 0.0;
  P.nrot = 0;
  int k0 = -1;
  for (int t = 0; t < r; ++t) {
    if (fabs(P.z[t]) <= tol) {
      P.z[t] = 0.0;
      continue;
    }
    if (k0 >= 0 && P.d[k0] - P.d[t] <= tol) {
      const double rho = hypot(P.z[k0], P.z[t]);
      const double c = P.z[k0] / rho, sn = P.z[t] / rho;
      P.z[k0] = rho;
      P.z[t] = 0.0;
      P.d[t] = P.d[k0];  // the pair is treated as one value, within tol
      P.rot_i[P.nrot] = k0;
      P.rot_j[P.nrot] = t;
      P.rot_c[P.nrot] = c;
      P.rot_s[P.nrot] = sn;
      ++P.nrot;
    } else {
      k0 = t;
    }
  }
  P.na = 0;
  for (int t = 0; t <= r; ++t)
    if (P.z[t] != 0.0) P.act[P.na++] = t;
  P.p_active = P.z[r] != 0.0;
  return tol;
}

// f(tau) and f'(tau) for the origin coordinate o (sigma = d_o + tau), over
// the active coordinates.
BSVD_FN void secular(const Problem& P, int o, double tau, double& f, double& df, double& fabs_sum) {
  const double dob = P.d[o];
  const double sig = dob + tau;
  double s = 1.0, ds = 0.0, a = 1.0;
  for (int k = 0; k < P.na; ++k) {
    const int t = P.act[k];
    const double del = (P.d[t] - dob) - tau;  // d_t - sigma
    const double sum = P.d[t] + sig;          // d_t + sigma
    const double q = P.z[t] / (del * sum);
    const double term = P.z[t] * q;
    s += term;
    a += fabs(term);
    ds += 2.0 * sig * q * q;
  }
  f = s;
  df = ds;
  fabs_sum = a;
}

// Root number k (0-based, descending) of the active problem.  Writes its
// origin coordinate and offset: sigma_k = d[o] + tau.
BSVD_FN void root(const Problem& P, int k, int& o_out, double& tau_out) {
  const int t = P.act[k];
  double lo, hi;
  int o;
  if (k == 0) {
    double zz = 0.0;
    for (int m = 0; m < P.na; ++m) zz += P.z[P.act[m]] * P.z[P.act[m]];
    o = t;
    lo = 0.0;
    hi = zz / (P.d[t] + sqrt(P.d[t] * P.d[t] + zz));
  } else {
    const int tp = P.act[k - 1];
    const double gap = P.d[tp] - P.d[t];
    double f, df, a;
    secular(P, t, 0.5 * gap, f, df, a);
    if (f >= 0.0) {
      o = t;
      lo = 0.0;
      hi = 0.5 * gap;
    } else {
      o = tp;
      lo = -0.5 * gap;
      hi = 0.0;
    }
  }
  // f < 0 at lo (or a pole there), f > 0 at hi (or a pole there)
  double tau = 0.5 * (lo + hi);
  for (int it = 0; it < kMaxNewton; ++it) {
    double f, df, a;
    secular(P, o, tau, f, df, a);
    if (f == 0.0 || fabs(f) <= kEps * a) break;
    if (f < 0.0)
      lo = tau;
    else
      hi = tau;
    if (hi - lo <= 2.0 * kEps * fmax(fabs(lo), fabs(hi))) break;
    double nt = tau - f / df;
    if (!(nt > lo && nt < hi)) {
      // bisection: geometric when the bracket spans orders of magnitude on
      // one side of zero, a step towards the pole when it is at zero
      if (lo > 0.0 && hi > 16.0 * lo)
        nt = sqrt(lo * hi);
      else if (hi < 0.0 && lo < 16.0 * hi)
        nt = -sqrt(lo * hi);
      else if (lo == 0.0 && hi > 0.0)
        nt = hi * (1.0 / 64.0);
      else if (hi == 0.0 && lo < 0.0)
        nt = lo * (1.0 / 64.0);
      else
        nt = 0.5 * (lo + hi);
    }
    if (nt == tau) break;
    tau = nt;
  }
  o_out = o;
  tau_out = tau;
}

// sigma_k - d_t and sigma_k + d_t from the stored (origin, tau).
BSVD_FN double minus_d(const Problem& P, int o, double tau, int t) { return (P.d[o] - P.d[t]) + tau; }
BSVD_FN double plus_d(const Problem& P, int o, double tau, int t) { return P.d[o] + tau + P.d[t]; }

// Loewner's formula for the active coordinate at position m: the z for which
// the computed roots are exact.
BSVD_FN double zhat(const Problem& P, int m, const int* org, const double* tau) {
  const int t = P.act[m];
  double prod = minus_d(P, org[m], tau[m], t) * plus_d(P, org[m], tau[m], t);
  for (int k = 0; k < P.na; ++k) {
    if (k == m) continue;
    const int u = P.act[k];
    const double num = minus_d(P, org[k], tau[k], t) * plus_d(P, org[k], tau[k], t);
    const double den = (P.d[u] - P.d[t]) * (P.d[u] + P.d[t]);
    prod *= num / den;
  }
  return copysign(sqrt(fabs(prod)), P.z[t]);
}

// Entry t of the unnormalised left and right vectors of root k, with zh the
// recomputed z of every coordinate (zero where deflated).
BSVD_FN void vec_entry(const Problem& P, const double* zh, int o, double tau, int t, double& ul, double& vr) {
  if (zh[t] == 0.0) {
    ul = 0.0;
    vr = (t == P.r) ? -1.0 : 0.0;
    return;
  }
  const double den = -(minus_d(P, o, tau, t) * plus_d(P, o, tau, t));  // d_t^2 - sigma^2
  ul = zh[t] / den;
  vr = (t == P.r) ? -1.0 : P.d[t] * zh[t] / den;
}

// Undo the deflation rotations on one column (coordinates < r), last first.
BSVD_FN void unrotate(const Problem& P, double* col, int stride) {
  for (int q = P.nrot - 1; q >= 0; --q) {
    const int i = P.rot_i[q], j = P.rot_j[q];
    const double c = P.rot_c[q], sn = P.rot_s[q];
    const double yi = col[(int64_t)i * stride], yj = col[(int64_t)j * stride];
    col[(int64_t)i * stride] = c * yi - sn * yj;
    col[(int64_t)j * stride] = sn * yi + c * yj;
  }
}

}  // namespace bsvd

namespace bsvd {

// Singular value of the candidate carried by coordinate t: the root whose gap
// starts at t when t is active (pos[t] = its index among the active
// coordinates), d_t when t is deflated.
BSVD_FN double cand_sigma(const Problem& P, const int* pos, const int* org, const double* tau, int t) {
  return pos[t] >= 0 ? P.d[org[pos[t]]] + tau[pos[t]] : P.d[t];
}

// Position of candidate t in the descending order of the n_cand candidates
// (coordinates 0..n_cand-1), ties by coordinate.
BSVD_FN int cand_rank(const double* sig, int n_cand, int t) {
  int rk = 0;
  for (int u = 0; u < n_cand; ++u) rk += (sig[u] > sig[t]) || (sig[u] == sig[t] && u < t);
  return rk;
}

// Left and right singular vectors of candidate t, normalised and rotated back
// to the coordinates of Q, written with the given element stride.
BSVD_FN void fill_column(const Problem& P, const double* zh, const int* pos, const int* org, const double* tau,
                         int t, double* ucol, double* vcol, int stride) {
  const int n = P.r + 1;
  if (pos[t] < 0) {
    for (int q = 0; q < n; ++q) {
      ucol[(int64_t)q * stride] = q == t ? 1.0 : 0.0;
      vcol[(int64_t)q * stride] = q == t ? 1.0 : 0.0;
    }
  } else {
    const int k = pos[t];
    double nu = 0.0, nv = 0.0;
    for (int q = 0; q < n; ++q) {
      double a, b;
      vec_entry(P, zh, org[k], tau[k], q, a, b);
      nu += a * a;
      nv += b * b;
    }
    const double iu = 1.0 / sqrt(nu), iv = 1.0 / sqrt(nv);
    for (int q = 0; q < n; ++q) {
      double a, b;
      vec_entry(P, zh, org[k], tau[k], q, a, b);
      ucol[(int64_t)q * stride] = a * iu;
      vcol[(int64_t)q * stride] = b * iv;
    }
  }
  unrotate(P, ucol, stride);
  unrotate(P, vcol, stride);
}

}  // namespace bsvd
