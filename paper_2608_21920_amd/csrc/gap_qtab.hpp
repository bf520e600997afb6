// Host construction of the quantum-spectrum tables (tubes with GAP_QUANTUM).
//
// Sect. 3.1 names the first-order QED synchrotron spectrum S(gamma, x) (and
// its Gaunt factor g_Q) and Sect. 3.2 the one-photon pair creation rate; the
// paper prints neither spectrum.  These are the textbook first-order forms:
//
//   photon energy fraction d = x/gamma of a lepton at chi, number spectrum
//     s(d) = (1 - d + 1/(1-d)) K_{2/3}(z) - Ki_{1/3}(z),  z = 2d/(3 chi (1-d));
//   electron energy fraction v of a pair from a photon at chi,
//     p(v) = (v/(1-v) + (1-v)/v) K_{2/3}(e) + Ki_{1/3}(e),  e = 2/(3 chi v(1-v)),
//
// with Ki_nu(z) = int_z^inf K_nu(t) dt.  The rates stay the paper's fits of
// T_syn and T_BW (eqs. tau_syn, tau_bw); only the energies are drawn from
// these spectra, so the mean recoil carries g_Q.  As chi -> 0, s dd becomes
// the classical spectrum (2 K_{2/3} - Ki_{1/3} = Ki_{5/3}) of the default
// sampler.
//
// Numerics: K_{2/3} and Ki_{1/3} from their integral representations over
// exp(-z cosh u) by the trapezoidal rule in u (step 1/8; geometric
// convergence), the distribution functions by fourth-order cumulative
// quadrature on fine grids (ln z for photons, w = 1/2 - v for pairs), and the
// inverse at each table node by cubic Hermite interpolation of the cumulative
// function between grid nodes.  Columns are built on all host threads.
#pragma once

#include <algorithm>
#include <cmath>
#include <mutex>
#include <thread>
#include <vector>

namespace gap {
namespace qtab {

constexpr double kPi = 3.14159265358979323846;

// Nodes of the u-quadrature: cosh u, cosh(2u/3), cosh(u/3)/cosh u, weights.
struct BesselNodes {
  std::vector<double> ch, c23, c13;
  BesselNodes() {
    const double h = 0.125;
    for (int i = 0; i * h <= 100.0; ++i) {
      const double u = i * h, c = std::cosh(u);
      const double wgt = (i == 0 ? 0.5 : 1.0) * h;
      ch.push_back(c);
      c23.push_back(wgt * std::cosh(2.0 * u / 3.0));
      c13.push_back(wgt * std::cosh(u / 3.0) / c);
    }
  }
  // K_{2/3}(z) exp(off), Ki_{1/3}(z) exp(off)
  void eval(double z, double off, double* k23, double* ki13) const {
    double a = 0.0, b = 0.0;
    for (size_t i = 0; i < ch.size(); ++i) {
      const double ex = z * ch[i] - off;
      if (ex > 740.0) break;
      const double e = std::exp(-ex);
      a += e * c23[i];
      b += e * c13[i];
    }
    *k23 = a;
    *ki13 = b;
  }
};

// Cumulative integrals of samples m[0..n] on a uniform grid of step h:
// left[k] = int_0^k, right[k] = int_k^n (fourth order inside, trapezoid at
// the two end intervals, where the integrands here are negligible).
inline void cumulate(const std::vector<double>& m, double h, std::vector<double>* left, std::vector<double>* right) {
  const size_t n = m.size() - 1;
  std::vector<double> seg(n);
  for (size_t k = 0; k < n; ++k) {
    if (k == 0 || k + 1 == n) seg[k] = 0.5 * h * (m[k] + m[k + 1]);
    else seg[k] = h / 24.0 * (-m[k - 1] + 13.0 * m[k] + 13.0 * m[k + 1] - m[k + 2]);
  }
  left->assign(n + 1, 0.0);
  right->assign(n + 1, 0.0);
  for (size_t k = 0; k < n; ++k) (*left)[k + 1] = (*left)[k] + seg[k];
  for (size_t k = n; k-- > 0;) (*right)[k] = (*right)[k + 1] + seg[k];
}

// Position x in [x_k, x_k + h] where a cumulative function with values c0,
// c1 and slopes m0, m1 at the ends reaches the value c (cubic Hermite,
// bisection-safeguarded Newton).  `rising` false: the function falls.
inline double hermite_solve(double x0, double h, double c0, double c1, double m0, double m1, double c, bool rising) {
  const double sg = rising ? 1.0 : -1.0;
  auto H = [&](double t, double* d) {
    const double t2 = t * t, t3 = t2 * t;
    const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + t, h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
    const double d00 = 6 * t2 - 6 * t, d10 = 3 * t2 - 4 * t + 1, d01 = -6 * t2 + 6 * t, d11 = 3 * t2 - 2 * t;
    *d = (d00 * c0 + d10 * h * m0 + d01 * c1 + d11 * h * m1);
    return h00 * c0 + h10 * h * m0 + h01 * c1 + h11 * h * m1;
  };
  double lo = 0.0, hi = 1.0;
  double t = (c1 != c0) ? std::min(std::max((c - c0) / (c1 - c0), 0.0), 1.0) : 0.5;
  for (int it = 0; it < 100; ++it) {
    double d;
    const double g = sg * (H(t, &d) - c);
    if (g > 0.0) hi = t; else lo = t;
    double tn = (d != 0.0) ? t - g / (sg * d) : 0.5 * (lo + hi);
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    if (std::fabs(tn - t) < 1e-14) { t = tn; break; }
    t = tn;
  }
  return x0 + t * h;
}

// One photon column: ln z at the rows of the table for lepton chi (0: classical).
inline void photon_column(const BesselNodes& bn, double chi, int nr, double alo, double ahi, double ylo, double yhi,
                          float* out) {
  const double slo = -72.0, shi = std::log(70.0);
  const int n = 12000;
  const double h = (shi - slo) / n;
  std::vector<double> m(n + 1);
  for (int k = 0; k <= n; ++k) {
    const double z = std::exp(slo + k * h);
    double k23, ki13;
    bn.eval(z, 0.0, &k23, &ki13);
    double dens;
    if (chi == 0.0) {
      dens = 2.0 * k23 - ki13;                              // Ki_{5/3}(z), per unit z
    } else {
      const double q = 2.0 + 3.0 * chi * z, omd = 2.0 / q;
      dens = ((omd + 1.0 / omd) * k23 - ki13) * (6.0 * chi / (q * q));
    }
    m[k] = dens * z;                                       // per unit ln z
  }
  std::vector<double> left, right;
  cumulate(m, h, &left, &right);
  // below the grid the spectrum per unit ln z falls as z^(1/3): the mass
  // there is 3 m[0]
  for (double& v : left) v += 3.0 * m[0];
  const double tot = left[n];
  // r <= 1/2: left cumulative reaches r tot
  for (int i = 0; i <= nr; ++i) {
    const double r = std::exp(alo + i * (ahi - alo) / nr);
    const double c = r * tot;
    const int k = (int)(std::upper_bound(left.begin(), left.end(), c) - left.begin()) - 1;
    const int kk = std::min(std::max(k, 0), n - 1);
    out[i] = (float)hermite_solve(slo + kk * h, h, left[kk], left[kk + 1], m[kk], m[kk + 1], c, true);
  }
  // r > 1/2: right cumulative (the tail) reaches (1 - r) tot = e^-y tot
  for (int i = 0; i <= nr; ++i) {
    const double y = ylo + i * (yhi - ylo) / nr;
    const double c = std::exp(-y) * tot;
    // right[] falls with k: first k with right[k+1] <= c
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (right[mid] > c) lo = mid; else hi = mid;
    }
    out[nr + 1 + i] = (float)hermite_solve(slo + lo * h, h, right[lo], right[lo + 1], -m[lo], -m[lo + 1], c, false);
  }
}

// One pair column: s = w sqrt((1+chi)/chi), w = 1/2 - v, at q = i/nr, r = q^4/2
// (dense rows toward the tail r -> 0, where v ~ 1/ln(1/r)).
inline void pair_column(const BesselNodes& bn, double chi, int nr, float* out) {
  const int n = 16000;
  const double h = 0.5 / n;
  const double off = 8.0 / (3.0 * chi);
  std::vector<double> m(n + 1);
  for (int k = 0; k <= n; ++k) {
    const double w = k * h;
    const double v = 0.5 - w, u = 0.5 + w;
    if (v <= 0.0) { m[k] = 0.0; continue; }
    const double e = 2.0 / (3.0 * chi * v * u);
    double k23, ki13;
    bn.eval(e, off, &k23, &ki13);
    m[k] = (v / u + u / v) * k23 + ki13;
  }
  std::vector<double> left, right;
  cumulate(m, h, &left, &right);
  const double half = left[n];
  const double sc = std::sqrt((1.0 + chi) / chi);
  for (int i = 0; i <= nr; ++i) {
    const double q = (double)i / nr, r = 0.5 * q * q * q * q;
    double w;
    if (i == 0) {
      w = 0.5;
    } else if (i == nr) {
      w = 0.0;
    } else {
      // the mass outside w (from w to 1/2, both sides) is 2 r of the whole:
      // right[k] = r' where r' = 2 r half (one side)
      const double c = 2.0 * r * half;
      int lo = 0, hi = n;
      while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (right[mid] > c) lo = mid; else hi = mid;
      }
      w = hermite_solve(lo * h, h, right[lo], right[lo + 1], -m[lo], -m[lo + 1], c, false);
    }
    out[i] = (float)(w * sc);
  }
}

struct Tables {
  std::vector<float> syn, bw;
};

// Built once per process (all columns on the host's threads).
inline const Tables& tables(int syn_cols, int syn_row, int syn_nr, double syn_chi_lo, int syn_per_dec, double alo,
                            double ahi, double ylo, double yhi, int bw_cols, int bw_nr, double bw_chi_lo,
                            int bw_per_dec) {
  static Tables t;
  static std::once_flag once;
  std::call_once(once, [&] {
    BesselNodes bn;
    t.syn.assign((size_t)syn_cols * syn_row, 0.0f);
    t.bw.assign((size_t)bw_cols * (bw_nr + 1), 0.0f);
    const int jobs = syn_cols + bw_cols;
    std::mutex mu;
    int next = 0;
    auto work = [&] {
      for (;;) {
        int j;
        {
          std::lock_guard<std::mutex> lk(mu);
          j = next++;
        }
        if (j >= jobs) return;
        if (j < syn_cols) {
          const double chi = j == 0 ? 0.0 : syn_chi_lo * std::pow(10.0, (double)(j - 1) / syn_per_dec);
          photon_column(bn, chi, syn_nr, alo, ahi, ylo, yhi, &t.syn[(size_t)j * syn_row]);
        } else {
          const int c = j - syn_cols;
          const double chi = bw_chi_lo * std::pow(10.0, (double)c / bw_per_dec);
          pair_column(bn, chi, bw_nr, &t.bw[(size_t)c * (bw_nr + 1)]);
        }
      }
    };
    const int nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int i = 1; i < nt; ++i) th.emplace_back(work);
    work();
    for (auto& x : th) x.join();
  });
  return t;
}

}  // namespace qtab
}  // namespace gap
