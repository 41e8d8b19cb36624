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
  double* da;      // [n] d and z of the active coordinates, contiguous (da[k] = d[act[k]])
  double* za;
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
    if (P.z[t] != 0.0) {
      P.da[P.na] = P.d[t];
      P.za[P.na] = P.z[t];
      P.act[P.na++] = t;
    }
  P.p_active = P.z[r] != 0.0;
  return tol;
}

// Partial sums of f(tau) - 1, f'(tau) and sum |terms| at sigma = dob + tau over
// the active coordinates k0, k0 + kstep, ... (a group of threads splits the
// sum and combines the parts).
BSVD_FN void secular_part(const Problem& P, double dob, double tau, int k0, int kstep, double& f, double& df,
                          double& fabs_sum) {
  const double sig = dob + tau;
  double s = 0.0, ds = 0.0, a = 0.0;
  const double* __restrict__ da = P.da;
  const double* __restrict__ za = P.za;
#pragma unroll 4
  for (int k = k0; k < P.na; k += kstep) {
    const double del = (da[k] - dob) - tau;  // d_t - sigma
    const double sum = da[k] + sig;          // d_t + sigma
    const double q = za[k] / (del * sum);
    const double term = za[k] * q;
    s += term;
    a += fabs(term);
    ds += 2.0 * sig * q * q;
  }
  f = s;
  df = ds;
  fabs_sum = a;
}

// Combines the partial sums of one group (nothing to do for one thread).
struct SoloSum {
  BSVD_FN void operator()(double&, double&, double&) const {}
};

// Root number k (0-based, descending) of the active problem, found by the
// group of threads that share k (each passes its k0 = rank in the group and
// kstep = group size, and `red` combines the group's partial sums).  Writes
// its origin (the nearer end of its gap) and offset: sigma_k = dorg + tau.
template <typename Red>
BSVD_FN void root_group(const Problem& P, int k, int k0, int kstep, Red red, double& dorg_out, double& tau_out) {
  double lo, hi, dob;
  if (k == 0) {
    double zz = 0.0, u = 0.0, w = 0.0;
    for (int m = k0; m < P.na; m += kstep) zz += P.za[m] * P.za[m];
    red(zz, u, w);
    dob = P.da[0];
    lo = 0.0;
    hi = zz / (dob + sqrt(dob * dob + zz));
  } else {
    const double gap = P.da[k - 1] - P.da[k];
    double f, df, a;
    secular_part(P, P.da[k], 0.5 * gap, k0, kstep, f, df, a);
    red(f, df, a);
    if (1.0 + f >= 0.0) {
      dob = P.da[k];
      lo = 0.0;
      hi = 0.5 * gap;
    } else {
      dob = P.da[k - 1];
      lo = -0.5 * gap;
      hi = 0.0;
    }
  }
  // f < 0 at lo (or a pole there), f > 0 at hi (or a pole there)
  double tau = 0.5 * (lo + hi);
  for (int it = 0; it < kMaxNewton; ++it) {
    double f, df, a;
    secular_part(P, dob, tau, k0, kstep, f, df, a);
    red(f, df, a);
    f += 1.0;
    a += 1.0;
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
  dorg_out = dob;
  tau_out = tau;
}

// One thread per root.
BSVD_FN void root(const Problem& P, int k, double& dorg_out, double& tau_out) {
  root_group(P, k, 0, 1, SoloSum{}, dorg_out, tau_out);
}

// sigma_k - d and sigma_k + d from the stored (origin, tau).
BSVD_FN double minus_d(double dorg, double tau, double d) { return (dorg - d) + tau; }
BSVD_FN double plus_d(double dorg, double tau, double d) { return dorg + tau + d; }

// Loewner's formula for the active coordinate at position m: the z for which
// the computed roots are exact.
BSVD_FN double zhat(const Problem& P, int m, const double* dorg, const double* tau) {
  const double dt = P.da[m];
  double prod = minus_d(dorg[m], tau[m], dt) * plus_d(dorg[m], tau[m], dt);
  for (int k = 0; k < P.na; ++k) {
    if (k == m) continue;
    const double du = P.da[k];
    const double num = minus_d(dorg[k], tau[k], dt) * plus_d(dorg[k], tau[k], dt);
    const double den = (du - dt) * (du + dt);
    prod *= num / den;
  }
  return copysign(sqrt(fabs(prod)), P.za[m]);
}

// Entry t of the unnormalised left and right vectors of the root
// (dorg, tau), with zh the recomputed z of every coordinate (zero where
// deflated).
BSVD_FN void vec_entry(const Problem& P, const double* zh, double dorg, double tau, int t, double& ul, double& vr) {
  if (zh[t] == 0.0) {
    ul = 0.0;
    vr = (t == P.r) ? -1.0 : 0.0;
    return;
  }
  const double dt = P.d[t];
  const double q = zh[t] / -(minus_d(dorg, tau, dt) * plus_d(dorg, tau, dt));  // z_t / (d_t^2 - sigma^2)
  ul = q;
  vr = (t == P.r) ? -1.0 : dt * q;
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
BSVD_FN double cand_sigma(const Problem& P, const int* pos, const double* dorg, const double* tau, int t) {
  return pos[t] >= 0 ? dorg[pos[t]] + tau[pos[t]] : P.d[t];
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
BSVD_FN void fill_column(const Problem& P, const double* zh, const int* pos, const double* dorg, const double* tau,
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
      vec_entry(P, zh, dorg[k], tau[k], q, a, b);
      ucol[(int64_t)q * stride] = a;
      vcol[(int64_t)q * stride] = b;
      nu += a * a;
      nv += b * b;
    }
    const double iu = 1.0 / sqrt(nu), iv = 1.0 / sqrt(nv);
    for (int q = 0; q < n; ++q) {
      ucol[(int64_t)q * stride] *= iu;
      vcol[(int64_t)q * stride] *= iv;
    }
  }
  unrotate(P, ucol, stride);
  unrotate(P, vcol, stride);
}

}  // namespace bsvd
