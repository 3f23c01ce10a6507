// icrs_oracle.cpp -- plain, slow FP64 CPU oracle of image-centred ray shooting (ICRS).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
// file: only the tests, the package's smoke check and the benchmark's CPU-baseline leg
// do.  It shares no code, header, table or constant generator with the HIP library.
//
// What it computes (paper: "microJAX", arXiv 2510.02639):
//   * lens equation and point-source magnification          -- Sec. 2.1, eqs. lens_eq, amp_point, detJ
//   * lens polynomial of degree N^2+1 (= 5(N-1) for N=2,3)    -- Sec. 2.1, eq. lens_eq_z
//   * Ehrlich-Aberth roots from a Cauchy-radius circle        -- Sec. 3.1 (EA update equation)
//   * root validation by substitution into the lens equation -- Sec. 2.1 (text after lens_eq_z)
//   * limb sampling, polar binning into sectors               -- Sec. 3.2 (limb-point equation, binning)
//   * fixed N_r x N_theta polar grid per sector, ray map      -- Sec. 2.2 (chi definition), Sec. 3.3
//   * row quadrature, cubic boundary crossing, uniform and
//     linear limb-darkened rules, radial sum, normalisation  -- App. A.1 and A.2
// Where the paper is silent or garbled the reading taken is stated at the spot; each
// reading also has a line in the repository's design notes.
//
// Plain scalar loops, std::complex<double>, no blocking or fusion.  Built with g++ -O2
// (no fast-math; x86-64 baseline has no FMA so nothing is contracted).

#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include <omp.h>

using cplx = std::complex<double>;

namespace {

constexpr double kPi = 3.14159265358979323846;

// Status bits of one epoch (shared meaning with the library, defined separately there).
enum : uint32_t {
  ST_ROOT_NONCONV = 1u,   // an EA solve hit its iteration cap
  ST_IMG_COUNT = 2u,      // an image count outside the allowed set after seeding
  ST_CAP_OVERFLOW = 4u,   // more sector candidates than the cap; pairs were merged
  ST_CLIP = 8u,           // inside rays still touch a sector edge after the retries
  ST_NAN = 16u,           // non-finite result
  ST_GIVEN = 64u,         // sectors were supplied by the caller
};

// ---------------------------------------------------------------------------------------
// O1: lens frame.  Sec. 2.1 (eq. lens_eq): fractional masses eps_i summing to 1, complex
// positions a_i, lengths in Einstein radii of the total mass.  Sec. 3.5 / Fig. 3 define the
// parameters: q = m2/m1, separation s on the real axis, origin at the M1-M2 barycentre;
// the third lens at (r3, psi) from the M1-M2 midpoint with q3 = m3/m1.
// Reading: the primary sits on the negative real axis.
// Parameter vector (doubles): [s, q, u0, alpha, t0, tE, rho, u1, q3, r3, psi].
// n_lens = 1 is a unit point lens at the origin, n_lens = 0 the identity map w = z
// (both used only as closed-form checks).
struct Lens {
  int n = 0;
  double eps[3] = {0, 0, 0};
  cplx a[3];
};

Lens make_lens(int n_lens, const double* p) {
  Lens L;
  L.n = n_lens;
  if (n_lens == 1) {
    L.eps[0] = 1.0;
    L.a[0] = cplx(0.0, 0.0);
  } else if (n_lens == 2) {
    const double s = p[0], q = p[1];
    L.eps[0] = 1.0 / (1.0 + q);
    L.eps[1] = q / (1.0 + q);
    L.a[0] = cplx(-q * s / (1.0 + q), 0.0);
    L.a[1] = cplx(s / (1.0 + q), 0.0);
  } else if (n_lens == 3) {
    const double s = p[0], q = p[1], q3 = p[8], r3 = p[9], psi = p[10];
    const double m = 1.0 + q + q3;
    L.eps[0] = 1.0 / m;
    L.eps[1] = q / m;
    L.eps[2] = q3 / m;
    L.a[0] = cplx(-q * s / (1.0 + q), 0.0);
    L.a[1] = cplx(s / (1.0 + q), 0.0);
    const cplx mid = 0.5 * (L.a[0] + L.a[1]);
    L.a[2] = mid + cplx(r3 * std::cos(psi), r3 * std::sin(psi));
  }
  return L;
}

// Eq. lens_eq: w = z - sum_i eps_i / (conj(z) - conj(a_i)).
cplx lens_map(const Lens& L, cplx z) {
  cplx w = z;
  for (int i = 0; i < L.n; ++i) w -= L.eps[i] / std::conj(z - L.a[i]);
  return w;
}

// kappa(z) = sum_i eps_i / (conj(z) - conj(a_i))^2; eq. detJ gives det J = 1 - |kappa|^2.
cplx kappa_of(const Lens& L, cplx z) {
  cplx k(0.0, 0.0);
  for (int i = 0; i < L.n; ++i) {
    const cplx d = std::conj(z - L.a[i]);
    k += L.eps[i] / (d * d);
  }
  return k;
}

// O2: source centre on a straight trajectory.  Sec. 3.5 names (t0, u0, tE, alpha) but not
// the sign conventions.  Reading: tau = (t - t0)/tE; the source moves along (cos a, sin a)
// and passes the origin at u0 * (-sin a, cos a) when t = t0.
cplx source_center(const double* p, double t) {
  const double u0 = p[2], alpha = p[3], t0 = p[4], tE = p[5];
  const double tau = (t - t0) / tE;
  return cplx(tau * std::cos(alpha) - u0 * std::sin(alpha), tau * std::sin(alpha) + u0 * std::cos(alpha));
}

// ---------------------------------------------------------------------------------------
// O4: lens polynomial, Sec. 2.1 eq. lens_eq_z.  The paper cites the degree 5(N-1) without
// printing coefficients.  Derivation used: conjugating eq. lens_eq gives conj(z) = G/H with
// H = prod_k (z - a_k), G = conj(w) H + sum_k eps_k prod_{j!=k} (z - a_j); putting this back
// into eq. lens_eq and clearing the denominators D_i = G - conj(a_i) H gives
//   P(z) = (z - w) prod_i D_i - H sum_i eps_i prod_{j!=i} D_j,
// of degree N^2 + 1 (5 for N = 2, 10 for N = 3) with leading coefficient prod_i(conj(w)-conj(a_i)).
using Poly = std::vector<cplx>;  // index = power of z

Poly pmul(const Poly& a, const Poly& b) {
  Poly c(a.size() + b.size() - 1, cplx(0.0, 0.0));
  for (size_t i = 0; i < a.size(); ++i)
    for (size_t j = 0; j < b.size(); ++j) c[i + j] += a[i] * b[j];
  return c;
}

Poly padd(const Poly& a, const Poly& b) {
  Poly c(std::max(a.size(), b.size()), cplx(0.0, 0.0));
  for (size_t i = 0; i < a.size(); ++i) c[i] += a[i];
  for (size_t i = 0; i < b.size(); ++i) c[i] += b[i];
  return c;
}

Poly pscale(const Poly& a, cplx s) {
  Poly c(a);
  for (auto& x : c) x *= s;
  return c;
}

Poly lens_polynomial(const Lens& L, cplx w) {
  const int n = L.n;
  Poly H{cplx(1.0, 0.0)};
  for (int k = 0; k < n; ++k) H = pmul(H, Poly{-L.a[k], cplx(1.0, 0.0)});
  Poly G = pscale(H, std::conj(w));
  for (int k = 0; k < n; ++k) {
    Poly Pk{cplx(1.0, 0.0)};
    for (int j = 0; j < n; ++j)
      if (j != k) Pk = pmul(Pk, Poly{-L.a[j], cplx(1.0, 0.0)});
    G = padd(G, pscale(Pk, cplx(L.eps[k], 0.0)));
  }
  std::vector<Poly> D(n);
  for (int i = 0; i < n; ++i) D[i] = padd(G, pscale(H, -std::conj(L.a[i])));
  Poly prodD{cplx(1.0, 0.0)};
  for (int i = 0; i < n; ++i) prodD = pmul(prodD, D[i]);
  Poly P = pmul(Poly{-w, cplx(1.0, 0.0)}, prodD);
  Poly S{cplx(0.0, 0.0)};
  for (int i = 0; i < n; ++i) {
    Poly Q{cplx(L.eps[i], 0.0)};
    for (int j = 0; j < n; ++j)
      if (j != i) Q = pmul(Q, D[j]);
    S = padd(S, Q);
  }
  P = padd(P, pscale(pmul(H, S), cplx(-1.0, 0.0)));
  P.resize(n * n + 2);  // degree n^2 + 1
  return P;
}

// ---------------------------------------------------------------------------------------
// O5: Ehrlich-Aberth, Sec. 3.1.  All estimates are updated together (Jacobi form) by
//   z_k <- z_k - ( P'(z_k)/P(z_k) - sum_{j!=k} 1/(z_k - z_j) )^{-1}.
// Start: uniformly on a circle of Cauchy radius R = 1 + max_{j<n} |b_j / b_n| (Sec. 3.1).
// Readings: circle centred at 0 with angular offset pi/(2n); the paper fixes an iteration
// count without giving it -- here each root stops on its own test (below), cap 500.
void horner(const Poly& P, cplx z, cplx* p, cplx* dp) {
  const int n = static_cast<int>(P.size()) - 1;
  cplx v = P[n], d(0.0, 0.0);
  for (int j = n - 1; j >= 0; --j) {
    d = d * z + v;
    v = v * z + P[j];
  }
  *p = v;
  *dp = d;
}

// With continue_from set, the iteration restarts from the estimates already in z (no Cauchy
// circle), runs at most cap iterations and stops a root on its step test only: the
// validation's last resort when the image count is still forbidden (see find_images).
bool ea_roots(const Poly& P, std::vector<cplx>& z, int* iters_out, bool continue_from = false, int cap = 500) {
  const int n = static_cast<int>(P.size()) - 1;
  if (!continue_from) {
    z.assign(n, cplx(0.0, 0.0));
    double R = 0.0;
    for (int j = 0; j < n; ++j) R = std::max(R, std::abs(P[j] / P[n]));
    R += 1.0;
    for (int k = 0; k < n; ++k) {
      const double ang = 2.0 * kPi * k / n + kPi / (2.0 * n);
      z[k] = cplx(R * std::cos(ang), R * std::sin(ang));
    }
  }
  const bool noise_stop = !continue_from;
  // A root is finished once its step is below 1e-14 max(1,|z|) or |P(z)| is down to the
  // rounding noise of evaluating P there, 8 n u sum_j |b_j| |z|^j with u = 2^-53 (clustered
  // roots never reach the first test).  Finished roots are no longer moved.
  std::vector<char> done(n, 0);
  std::vector<cplx> step(n);
  for (int it = 0; it < cap; ++it) {
    for (int k = 0; k < n; ++k) {
      step[k] = cplx(0.0, 0.0);
      if (done[k]) continue;
      cplx p, dp;
      horner(P, z[k], &p, &dp);
      double noise = 0.0;
      const double az = std::abs(z[k]);
      for (int j = n; j >= 0; --j) noise = noise * az + std::abs(P[j]);
      noise *= 8.0 * n * 1.1102230246251565e-16;
      // P(z) exactly zero: z is a root, its correction (P/P') / (1 - (P/P') S) is zero
      if (p == cplx(0.0, 0.0) || (noise_stop && std::abs(p) <= noise)) {
        done[k] = 1;
        continue;
      }
      cplx rep(0.0, 0.0);
      for (int j = 0; j < n; ++j)
        if (j != k && z[k] != z[j]) rep += 1.0 / (z[k] - z[j]);
      const cplx den = dp / p - rep;
      step[k] = (den == cplx(0.0, 0.0)) ? cplx(0.0, 0.0) : 1.0 / den;
    }
    bool all = true;
    for (int k = 0; k < n; ++k) {
      if (done[k]) continue;
      z[k] -= step[k];
      if (std::abs(step[k]) <= 1e-14 * std::max(1.0, std::abs(z[k]))) done[k] = 1;
      all = all && done[k];
    }
    if (all) {
      if (iters_out) *iters_out = it + 1;
      return true;
    }
  }
  if (iters_out) *iters_out = cap;
  return false;
}

// ---------------------------------------------------------------------------------------
// O6: validation, Sec. 2.1 ("each root ... must be validated by substituting it back").
// Reading of the tolerance: every root is polished by Newton steps on the lens
// equation itself (with F = lens_map(z) - w and kappa as above, the step solving
// dz + kappa conj(dz) = -F is dz = (kappa conj(F) - F) / (1 - |kappa|^2)), kept when
// |F| <= 1e-10 afterwards, and dropped as a duplicate within 1e-9 max(1,|z|) of a kept one.
// Steps stop once a step is below 1e-14 max(1,|z|).  After 8 steps a root goes on, to 24 at
// most, while it is within the residual bound or its |F| at least halves per step: a
// spurious root of the polynomial can wander into an image's basin and stop within the
// residual bound yet outside the duplicate radius, which would count that image twice; and a
// root of a tight cluster next to a low-mass lens, accurate only to the cluster's
// conditioning (~1e-5), needs more than 8 Newton steps to reach its image across the nearby
// critical curve, and a fixed cap there drops a true image.
// An image count outside {N+1, N+3, ..., 5(N-1)} triggers one extra pass seeded next to
// each lens (z = a_k - eps_k / conj(w' - a_k), w' = w shifted by the other lenses'
// deflection at a_k -- the leading-order image near a lens); a count still outside the
// set raises ST_IMG_COUNT.
cplx polish(const Lens& L, cplx w, cplx z) {
  double f_prev = std::numeric_limits<double>::infinity();
  for (int s = 0; s < 24; ++s) {
    const cplx F = lens_map(L, z) - w;
    const double f = std::abs(F);
    if (s >= 8 && !(f <= 1e-10) && !(f <= 0.5 * f_prev)) break;
    f_prev = f;
    const cplx k = kappa_of(L, z);
    const double den = 1.0 - std::norm(k);
    if (den == 0.0 || !std::isfinite(den)) break;
    const cplx dz = (k * std::conj(F) - F) / den;
    z += dz;
    if (std::abs(dz) <= 1e-14 * std::max(1.0, std::abs(z))) break;
  }
  return z;
}

bool count_ok(int n_lens, int count) {
  if (n_lens == 0) return count == 1;
  if (n_lens == 1) return count == 2;
  const int lo = n_lens + 1, hi = 5 * (n_lens - 1);
  return count >= lo && count <= hi && ((count - lo) % 2 == 0);
}

void try_accept(const Lens& L, cplx w, cplx z0, std::vector<cplx>& out) {
  const cplx z = polish(L, w, z0);
  const double res = std::abs(lens_map(L, z) - w);
  if (!(res <= 1e-10)) return;
  for (const cplx& y : out)
    if (std::abs(z - y) <= 1e-9 * std::max(1.0, std::abs(z))) return;
  out.push_back(z);
}

// Images of the point source at w.  Returns status bits (ST_ROOT_NONCONV, ST_IMG_COUNT).
uint32_t find_images(const Lens& L, cplx w, std::vector<cplx>& images) {
  uint32_t st = 0;
  images.clear();
  const Poly P = lens_polynomial(L, w);
  std::vector<cplx> roots;
  int iters = 0;
  if (!ea_roots(P, roots, &iters)) st |= ST_ROOT_NONCONV;
  auto validate = [&]() {
    images.clear();
    for (const cplx& r : roots) try_accept(L, w, r, images);
    if (!count_ok(L.n, static_cast<int>(images.size()))) {
      for (int k = 0; k < L.n; ++k) {
        cplx wk = w;
        for (int j = 0; j < L.n; ++j)
          if (j != k) wk += L.eps[j] / std::conj(L.a[k] - L.a[j]);
        try_accept(L, w, L.a[k] - L.eps[k] / std::conj(wk - L.a[k]), images);
      }
    }
    return count_ok(L.n, static_cast<int>(images.size()));
  };
  if (!validate()) {
    // Two estimates that stopped on the rounding-noise test inside one root's neighbourhood
    // (a tight cluster of roots next to a low-mass lens) leave a root, and its image, unfound.
    // Last resort: continue the simultaneous iteration from the current estimates with the
    // step test only (the repulsion term of Sec. 3.1 then separates the pair), at most 100
    // iterations, and validate again.
    int it2 = 0;
    ea_roots(P, roots, &it2, true, 100);
    if (!validate()) st |= ST_IMG_COUNT;
  }
  return st;
}

// ---------------------------------------------------------------------------------------
// O8: sectors, Sec. 3.2.  The paper bins image-limb points in polar (r, theta) separately in
// r and theta, forms candidate (r-bin x theta-bin) sectors, keeps occupied ones, merges
// periodic/overlapping ones, caps the count by the maximum number of images, and sets
// bounds from min/max of enclosed points plus a safety margin.  It gives none of the
// constants.  Readings taken:
//   polar origin = frame origin; 64 theta bins on (-pi, pi]; r bins of width
//   max((r_max - r_min)/32, 2 rho) from r_min (32 bins); a run = occupied bins joined across
//   gaps of at most one empty bin (theta circular; no gap of >= 2 empty bins = full ring);
//   candidate = (r-run, theta-run) pair holding >= 1 point; bounds = member min/max (theta
//   unwrapped within its run); margin per side 0.1 x extent + floor (rho/100 in r,
//   rho/(100 r_mid) in theta), r_lo >= 0, theta extent >= 2 pi -> full ring; merge any two
//   sectors overlapping in r and circularly in theta into their bounding box, to a fixpoint;
//   cap at 5(N-1) by merging the pair of least union area; sort by (theta_lo, r_lo).
struct Sector {
  double r_lo, r_hi, th_lo, th_hi;
  bool periodic;
};

constexpr int kBinsTheta = 64;
constexpr int kBinsR = 32;

void normalise_theta(Sector& s) {
  if (s.periodic || s.th_hi - s.th_lo >= 2.0 * kPi) {
    s.periodic = true;
    s.th_lo = -kPi;
    s.th_hi = kPi;
    return;
  }
  while (s.th_lo < -kPi) {
    s.th_lo += 2.0 * kPi;
    s.th_hi += 2.0 * kPi;
  }
  while (s.th_lo >= kPi) {
    s.th_lo -= 2.0 * kPi;
    s.th_hi -= 2.0 * kPi;
  }
}

// Shift (k in {-1,0,1}) of b's theta interval by 2 pi k that makes it overlap a; 2 if none.
int theta_overlap_shift(const Sector& a, const Sector& b) {
  if (a.periodic || b.periodic) return 0;
  for (int k = -1; k <= 1; ++k) {
    const double lo = b.th_lo + 2.0 * kPi * k, hi = b.th_hi + 2.0 * kPi * k;
    if (lo <= a.th_hi && a.th_lo <= hi) return k;
  }
  return 2;
}

bool overlaps(const Sector& a, const Sector& b) {
  if (!(a.r_lo <= b.r_hi && b.r_lo <= a.r_hi)) return false;
  return theta_overlap_shift(a, b) != 2;
}

Sector union_of(const Sector& a, const Sector& b) {
  Sector u;
  u.r_lo = std::min(a.r_lo, b.r_lo);
  u.r_hi = std::max(a.r_hi, b.r_hi);
  u.periodic = a.periodic || b.periodic;
  if (u.periodic) {
    u.th_lo = -kPi;
    u.th_hi = kPi;
    return u;
  }
  int k = theta_overlap_shift(a, b);
  if (k == 2) {  // disjoint in theta (only in the cap step): join across the shorter gap
    double best = 1e300;
    for (int kk = -1; kk <= 1; ++kk) {
      const double lo = std::min(a.th_lo, b.th_lo + 2.0 * kPi * kk);
      const double hi = std::max(a.th_hi, b.th_hi + 2.0 * kPi * kk);
      if (hi - lo < best) {
        best = hi - lo;
        k = kk;
      }
    }
  }
  u.th_lo = std::min(a.th_lo, b.th_lo + 2.0 * kPi * k);
  u.th_hi = std::max(a.th_hi, b.th_hi + 2.0 * kPi * k);
  normalise_theta(u);
  return u;
}

double polar_area(const Sector& s) { return 0.5 * (s.r_hi * s.r_hi - s.r_lo * s.r_lo) * (s.th_hi - s.th_lo); }

void merge_fixpoint(std::vector<Sector>& S) {
  bool changed = true;
  while (changed) {
    changed = false;
    for (size_t i = 0; i < S.size() && !changed; ++i)
      for (size_t j = i + 1; j < S.size() && !changed; ++j)
        if (overlaps(S[i], S[j])) {
          S[i] = union_of(S[i], S[j]);
          S.erase(S.begin() + j);
          changed = true;
        }
  }
}

void sort_sectors(std::vector<Sector>& S) {
  std::stable_sort(S.begin(), S.end(), [](const Sector& a, const Sector& b) {
    if (a.th_lo != b.th_lo) return a.th_lo < b.th_lo;
    return a.r_lo < b.r_lo;
  });
}

// Circular runs over nb bins; returns (start, length) pairs, or one run of length nb.
std::vector<std::pair<int, int>> circular_runs(const std::vector<int>& occ) {
  const int nb = static_cast<int>(occ.size());
  std::vector<std::pair<int, int>> runs;
  int n_occ = 0;
  for (int b = 0; b < nb; ++b) n_occ += occ[b] ? 1 : 0;
  if (n_occ == 0) return runs;
  // a gap of >= 2 empty bins breaks a run; find the first bin that follows such a gap
  int start = -1;
  for (int b = 0; b < nb; ++b) {
    if (occ[b] && !occ[(b - 1 + nb) % nb] && !occ[(b - 2 + nb) % nb]) {
      start = b;
      break;
    }
  }
  if (start < 0) {  // no gap of two empty bins anywhere: one full ring
    runs.push_back({0, nb});
    return runs;
  }
  int b = start;
  int visited = 0;
  while (visited < nb) {
    if (!occ[b]) {
      ++b;
      b %= nb;
      ++visited;
      continue;
    }
    const int s = b;
    int last = b;  // last occupied bin of this run
    int len = 1;
    ++b;
    b %= nb;
    ++visited;
    while (visited < nb) {
      if (occ[b]) {
        last = b;
      } else if (!occ[(b + 1) % nb]) {
        break;  // two empty bins in a row end the run
      }
      ++b;
      b %= nb;
      ++visited;
    }
    len = (last - s + nb) % nb + 1;
    runs.push_back({s, len});
  }
  return runs;
}

std::vector<std::pair<int, int>> linear_runs(const std::vector<int>& occ) {
  const int nb = static_cast<int>(occ.size());
  std::vector<std::pair<int, int>> runs;
  int b = 0;
  while (b < nb) {
    if (!occ[b]) {
      ++b;
      continue;
    }
    const int s = b;
    int last = b;
    ++b;
    while (b < nb) {
      if (occ[b]) {
        last = b;
      } else if (b + 1 >= nb || !occ[b + 1]) {
        break;
      }
      ++b;
    }
    runs.push_back({s, last - s + 1});
    b = last + 1;
  }
  return runs;
}

uint32_t build_sectors(const std::vector<double>& r, const std::vector<double>& th, double rho, int cap,
                       std::vector<Sector>& out) {
  uint32_t st = 0;
  out.clear();
  const size_t P = r.size();
  if (P == 0) return st;
  // theta bins on (-pi, pi]
  const double wth = 2.0 * kPi / kBinsTheta;
  std::vector<int> tbin(P), occ_t(kBinsTheta, 0);
  for (size_t p = 0; p < P; ++p) {
    int b = static_cast<int>(std::floor((th[p] + kPi) / wth));
    b = std::min(std::max(b, 0), kBinsTheta - 1);
    tbin[p] = b;
    occ_t[b] = 1;
  }
  // r bins
  double rmin = r[0], rmax = r[0];
  for (size_t p = 1; p < P; ++p) {
    rmin = std::min(rmin, r[p]);
    rmax = std::max(rmax, r[p]);
  }
  const double wr = std::max((rmax - rmin) / kBinsR, 2.0 * rho);
  std::vector<int> rbin(P), occ_r(kBinsR, 0);
  for (size_t p = 0; p < P; ++p) {
    int b = static_cast<int>(std::floor((r[p] - rmin) / wr));
    b = std::min(std::max(b, 0), kBinsR - 1);
    rbin[p] = b;
    occ_r[b] = 1;
  }
  const auto truns = circular_runs(occ_t);
  const auto rruns = linear_runs(occ_r);
  std::vector<Sector> cand;
  for (const auto& rr : rruns) {
    for (const auto& tr : truns) {
      const bool full = tr.second >= kBinsTheta;
      bool any = false;
      Sector s{0, 0, 0, 0, full};
      for (size_t p = 0; p < P; ++p) {
        if (rbin[p] < rr.first || rbin[p] >= rr.first + rr.second) continue;
        const int off = (tbin[p] - tr.first + kBinsTheta) % kBinsTheta;
        if (!full && off >= tr.second) continue;
        const double thu = (tbin[p] >= tr.first) ? th[p] : th[p] + 2.0 * kPi;
        if (!any) {
          s.r_lo = s.r_hi = r[p];
          s.th_lo = s.th_hi = thu;
          any = true;
        } else {
          s.r_lo = std::min(s.r_lo, r[p]);
          s.r_hi = std::max(s.r_hi, r[p]);
          s.th_lo = std::min(s.th_lo, thu);
          s.th_hi = std::max(s.th_hi, thu);
        }
      }
      if (!any) continue;
      // safety margins
      const double r_mid = 0.5 * (s.r_lo + s.r_hi);
      const double mr = 0.1 * (s.r_hi - s.r_lo) + rho / 100.0;
      const double mt = 0.1 * (s.th_hi - s.th_lo) + rho / (100.0 * r_mid);
      s.r_lo = std::max(s.r_lo - mr, 0.0);
      s.r_hi = s.r_hi + mr;
      if (!full) {
        s.th_lo -= mt;
        s.th_hi += mt;
      }
      normalise_theta(s);
      cand.push_back(s);
    }
  }
  merge_fixpoint(cand);
  while (static_cast<int>(cand.size()) > cap) {
    st |= ST_CAP_OVERFLOW;
    size_t bi = 0, bj = 1;
    double best = 1e300;
    for (size_t i = 0; i < cand.size(); ++i)
      for (size_t j = i + 1; j < cand.size(); ++j) {
        const double a = polar_area(union_of(cand[i], cand[j]));
        if (a < best) {
          best = a;
          bi = i;
          bj = j;
        }
      }
    cand[bi] = union_of(cand[bi], cand[bj]);
    cand.erase(cand.begin() + bj);
    merge_fixpoint(cand);
  }
  sort_sectors(cand);
  out = cand;
  return st;
}

// ---------------------------------------------------------------------------------------
// O9-O11: ray shooting and quadrature on one sector, Sec. 3.3 and App. A.
//
// Grid (Sec. 3.3): N_r x N_theta nodes; reading: cell-centred, r_i = r_lo + (i+1/2) dr,
// theta_l = theta_lo + (l+1/2) dtheta, so r_i dr dtheta is the exact annular-cell area.
// Each node z = r_i e^{i theta_l} is mapped by eq. lens_eq; d = |w - w_c|; chi = [d < rho]
// (Sec. 2.2, strict).
//
// Surface brightness, App. A.2: I(x) = I0 [1 - u1 (1 - sqrt(1 - x^2))], x = d/rho, with
// I0 = 3 / (pi (3 - u1)) (read as 3 divided by pi(3 - u1): it normalises the flux to one).
//
// Boundary weights, App. A.2: each inside node owns [theta_l - dtheta/2, theta_l + dtheta/2].
// Reading of the garbled delta_enter: delta is the distance from the crossing to the node in
// units of dtheta (in [0,1]), so a boundary node owns (delta + 1/2) dtheta of its row.  Node
// weight W = 1 + sum over the sides whose neighbour is outside of (f(delta_side) - 1); for a
// node with one outside neighbour this is exactly f(delta) (entering/exiting classes), for a
// fully enclosed node 1.  f is the App. A.2 hybrid for u1 > 0 with b(delta) =
// (2/3) sqrt(1 + 1/(2 delta)); the uniform source (u1 = 0) uses f(delta) = delta + 1/2, the
// node-centred form of App. A.1.  delta_c is not given; reading: 0.1.
//
// Crossing (App. A.1/A.2): on the bracket (p, p+1), t = (theta - theta_p)/dtheta, the cubic
// Lagrange interpolant L(t) of d through t = -1, 0, 1, 2 (nodes p-1..p+2) is solved for
// L(t) = rho by bisection on [0,1] (60 halvings, left half kept on an exact hit).  At a
// non-periodic edge where p-1 or p+2 does not exist, the linear interpolant is used.  A
// neighbour beyond a non-periodic edge counts as outside with delta = 1/2 and is reported.
//
// Row sum A_i = r_i dtheta sum_l I_l chi_l W_l; sector sum dr sum_i A_i (App. A.1);
// magnification = sum over sectors / rho^2 with I normalised (App. A.2).
double lagrange4(const double d[4], double t) {
  const double tm1 = t + 1.0, t0 = t, t1 = t - 1.0, t2 = t - 2.0;
  return d[0] * (-(t0 * t1 * t2) / 6.0) + d[1] * (tm1 * t1 * t2 / 2.0) + d[2] * (-(tm1 * t0 * t2) / 2.0) +
         d[3] * (tm1 * t0 * t1 / 6.0);
}

// Solve for the crossing in [0,1].  cubic != 0: d4 = {d_{p-1}, d_p, d_{p+1}, d_{p+2}};
// cubic == 0: linear between d4[1] and d4[2].
double crossing_t(const double d4[4], int cubic, double rho) {
  if (!cubic) {
    const double den = d4[2] - d4[1];
    double t = (den == 0.0) ? 0.5 : (rho - d4[1]) / den;
    return std::min(std::max(t, 0.0), 1.0);
  }
  double a = 0.0, b = 1.0;
  const bool in_a = (lagrange4(d4, a) - rho) < 0.0;
  for (int it = 0; it < 60; ++it) {
    const double m = 0.5 * (a + b);
    const double g = lagrange4(d4, m) - rho;
    if (g == 0.0) {
      b = m;
    } else if ((g < 0.0) == in_a) {
      a = m;
    } else {
      b = m;
    }
  }
  return 0.5 * (a + b);
}

double brightness(double x, double u1) {
  const double I0 = 3.0 / (kPi * (3.0 - u1));
  const double c = 1.0 - x * x;
  return I0 * (1.0 - u1 * (1.0 - std::sqrt(c > 0.0 ? c : 0.0)));
}

double edge_factor(double delta, double u1, double delta_c) {
  if (u1 == 0.0) return delta + 0.5;
  if (delta >= delta_c && delta > 0.0) return (0.5 + delta) * (2.0 / 3.0) * std::sqrt(1.0 + 1.0 / (2.0 * delta));
  return (2.0 / 3.0) * delta + 0.5;
}

// Clip flags of one sector: bit0 r_lo row, bit1 r_hi row, bit2 theta_lo column, bit3 theta_hi column.
double sector_flux(const Lens& L, cplx wc, double rho, double u1, double delta_c, int nr, int nth, const Sector& S,
                   int* clip_flags) {
  const double dr = (S.r_hi - S.r_lo) / nr;
  const double dth = (S.th_hi - S.th_lo) / nth;
  std::vector<double> d(nth);
  std::vector<char> in(nth);
  double total = 0.0;
  int clip = 0;
  for (int i = 0; i < nr; ++i) {
    const double ri = S.r_lo + (i + 0.5) * dr;
    bool any_in = false;
    for (int l = 0; l < nth; ++l) {
      const double th = S.th_lo + (l + 0.5) * dth;
      const cplx z(ri * std::cos(th), ri * std::sin(th));
      const cplx w = lens_map(L, z);
      d[l] = std::abs(w - wc);
      in[l] = d[l] < rho;
      any_in = any_in || in[l];
    }
    if (!any_in) continue;
    if (i == 0 && S.r_lo > 0.0) clip |= 1;
    if (i == nr - 1) clip |= 2;
    double row = 0.0;
    for (int l = 0; l < nth; ++l) {
      if (!in[l]) continue;
      double W = 1.0;
      // left side: crossing in (theta_{l-1}, theta_l), bracket p = l-1, delta = 1 - t
      if (l == 0 && !S.periodic) {
        clip |= 4;
        W += edge_factor(0.5, u1, delta_c) - 1.0;
      } else {
        const int lm = (l - 1 + nth) % nth;
        if (!in[lm]) {
          const int p = lm;
          double st[4];
          int cubic = 1;
          for (int j = -1; j <= 2; ++j) {
            int idx = p + j;
            if (S.periodic) {
              idx = (idx % nth + nth) % nth;
            } else if (idx < 0 || idx >= nth) {
              cubic = 0;
              idx = std::min(std::max(idx, 0), nth - 1);
            }
            st[j + 1] = d[idx];
          }
          const double t = crossing_t(st, cubic, rho);
          W += edge_factor(1.0 - t, u1, delta_c) - 1.0;
        }
      }
      // right side: crossing in (theta_l, theta_{l+1}), bracket p = l, delta = t
      if (l == nth - 1 && !S.periodic) {
        clip |= 8;
        W += edge_factor(0.5, u1, delta_c) - 1.0;
      } else {
        const int lp = (l + 1) % nth;
        if (!in[lp]) {
          const int p = l;
          double st[4];
          int cubic = 1;
          for (int j = -1; j <= 2; ++j) {
            int idx = p + j;
            if (S.periodic) {
              idx = (idx % nth + nth) % nth;
            } else if (idx < 0 || idx >= nth) {
              cubic = 0;
              idx = std::min(std::max(idx, 0), nth - 1);
            }
            st[j + 1] = d[idx];
          }
          const double t = crossing_t(st, cubic, rho);
          W += edge_factor(t, u1, delta_c) - 1.0;
        }
      }
      row += brightness(d[l] / rho, u1) * W;
    }
    total += ri * dth * row * dr;
  }
  if (clip_flags) *clip_flags = clip;
  return total;
}

// O12: clip certificate (not in the paper; the paper's safety margin has no check).
// A sector whose inside rays touch an edge row/column is widened by half its extent on that
// side, the list is merged again, and the epoch is recomputed; at most max_retries times.
void widen(Sector& s, int clip) {
  const double er = s.r_hi - s.r_lo;
  if (clip & 1) s.r_lo = std::max(s.r_lo - 0.5 * er, 0.0);
  if (clip & 2) s.r_hi += 0.5 * er;
  if (!s.periodic) {
    const double et = s.th_hi - s.th_lo;
    if (clip & 4) s.th_lo -= 0.5 * et;
    if (clip & 8) s.th_hi += 0.5 * et;
    normalise_theta(s);
  }
}

// The retry step: every flagged sector widened on its flagged sides, then the list merged to
// a fixpoint and sorted again (widened sectors may now overlap their neighbours).
void retry_sectors(std::vector<Sector>& sectors, const std::vector<int>& clips) {
  for (size_t s = 0; s < sectors.size(); ++s)
    if (clips[s]) widen(sectors[s], clips[s]);
  merge_fixpoint(sectors);
  sort_sectors(sectors);
}

struct Config {
  int n_limb, n_r, n_theta, max_retries;
  double delta_c;
};

// One epoch end to end.  Returns the magnification; fills status and the final sector list.
double epoch_magnification(const Lens& L, const double* p, double t, const Config& cfg, uint32_t* status,
                           std::vector<Sector>& sectors, double* a_ps, int* n_img_center) {
  uint32_t st = 0;
  const double rho = p[6], u1 = p[7];
  const cplx wc = source_center(p, t);
  // centre images: point-source magnification, eq. amp_point with eq. detJ
  std::vector<cplx> img;
  st |= find_images(L, wc, img);
  double aps = 0.0;
  for (const cplx& z : img) aps += 1.0 / std::abs(1.0 - std::norm(kappa_of(L, z)));
  if (a_ps) *a_ps = aps;
  if (n_img_center) *n_img_center = static_cast<int>(img.size());
  // O3: limb points w_k = w_c + rho e^{2 pi i k / N_limb}, k = 0..N_limb-1 (Sec. 3.2; the
  // printed exponent drops k -- read as the k-th of N_limb equally spaced points, phase 0).
  std::vector<double> rr, tt;
  for (int k = 0; k < cfg.n_limb; ++k) {
    const double ph = 2.0 * kPi * k / cfg.n_limb;
    const cplx w = wc + cplx(rho * std::cos(ph), rho * std::sin(ph));
    st |= find_images(L, w, img);
    for (const cplx& z : img) {
      rr.push_back(std::abs(z));
      tt.push_back(std::atan2(z.imag(), z.real()));
    }
  }
  const int cap = (L.n >= 2) ? 5 * (L.n - 1) : 2;
  st |= build_sectors(rr, tt, rho, cap, sectors);
  double flux = 0.0;
  for (int attempt = 0;; ++attempt) {
    flux = 0.0;
    std::vector<int> clips(sectors.size(), 0);
    bool any = false;
    for (size_t s = 0; s < sectors.size(); ++s) {
      flux += sector_flux(L, wc, rho, u1, cfg.delta_c, cfg.n_r, cfg.n_theta, sectors[s], &clips[s]);
      any = any || clips[s] != 0;
    }
    if (!any) break;
    if (attempt >= cfg.max_retries) {
      st |= ST_CLIP;
      break;
    }
    retry_sectors(sectors, clips);
  }
  const double mag = flux / (rho * rho);
  if (!std::isfinite(mag)) st |= ST_NAN;
  *status = st;
  return mag;
}

// ---------------------------------------------------------------------------------------
// O13: gradients on the frozen structure (not in the paper, which uses forward-mode AD with
// a sigmoid surrogate for chi).  The sector boxes, the inside/outside pattern chi, each
// crossing's stencil and each edge factor's branch are taken from a reference evaluation;
// with them fixed, the magnification is a smooth function of the parameters.  Its
// derivative is computed by forward-mode dual numbers with one tangent per parameter; the
// crossing position, found by bisection on values, gets its tangent from the implicit
// function theorem on L(t) = rho:  dt = (drho - sum_j l_j(t) dd_j) / L'(t).
constexpr int kNT = 11;

struct Dual {
  double v = 0.0;
  double d[kNT] = {};
  Dual() = default;
  Dual(double x) : v(x) {}  // NOLINT: constants promote implicitly
};
Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v);
  for (int k = 0; k < kNT; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v);
  for (int k = 0; k < kNT; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
Dual operator-(const Dual& a) { return Dual(0.0) - a; }
Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v);
  for (int k = 0; k < kNT; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int k = 0; k < kNT; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
Dual dsqrt(const Dual& a) {
  Dual r(std::sqrt(a.v));
  for (int k = 0; k < kNT; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
  return r;
}
Dual dsin(const Dual& a) {
  Dual r(std::sin(a.v));
  for (int k = 0; k < kNT; ++k) r.d[k] = a.d[k] * std::cos(a.v);
  return r;
}
Dual dcos(const Dual& a) {
  Dual r(std::cos(a.v));
  for (int k = 0; k < kNT; ++k) r.d[k] = -a.d[k] * std::sin(a.v);
  return r;
}
double val(double x) { return x; }
double val(const Dual& x) { return x.v; }
double dsqrt(double x) { return std::sqrt(x); }
double dsin(double x) { return std::sin(x); }
double dcos(double x) { return std::cos(x); }

template <class S>
struct LensT {
  int n = 0;
  S eps[3];
  S ax[3], ay[3];
};

// the frame of make_lens(), in scalar type S
template <class S>
LensT<S> make_lens_t(int n_lens, const S* p) {
  LensT<S> L;
  L.n = n_lens;
  if (n_lens == 1) {
    L.eps[0] = S(1.0);
    L.ax[0] = S(0.0);
    L.ay[0] = S(0.0);
  } else if (n_lens >= 2) {
    const S s = p[0], q = p[1];
    const S q3 = (n_lens == 3) ? p[8] : S(0.0);
    const S pair = S(1.0) + q;
    const S m = pair + q3;
    L.eps[0] = S(1.0) / m;
    L.eps[1] = q / m;
    L.ax[0] = -(q * s) / pair;
    L.ax[1] = s / pair;
    L.ay[0] = S(0.0);
    L.ay[1] = S(0.0);
    if (n_lens == 3) {
      L.eps[2] = q3 / m;
      const S mid = S(0.5) * (L.ax[0] + L.ax[1]);
      L.ax[2] = mid + p[9] * dcos(p[10]);
      L.ay[2] = p[9] * dsin(p[10]);
    }
  }
  return L;
}

template <class S>
void source_center_t(const S* p, double t, S* wx, S* wy) {
  const S tau = (S(t) - p[4]) / p[5];
  *wx = tau * dcos(p[3]) - p[2] * dsin(p[3]);
  *wy = tau * dsin(p[3]) + p[2] * dcos(p[3]);
}

// d = |lens_map(z) - w_c| for a grid node z (no tangent)
template <class S>
S node_distance(const LensT<S>& L, double zx, double zy, const S& wx, const S& wy) {
  S ux = S(zx) - wx, uy = S(zy) - wy;
  for (int k = 0; k < L.n; ++k) {
    const S dx = S(zx) - L.ax[k], dy = S(zy) - L.ay[k];
    const S inv = L.eps[k] / (dx * dx + dy * dy);  // eps / conj(z - a) = eps (z - a) / |z - a|^2
    ux = ux - inv * dx;
    uy = uy - inv * dy;
  }
  return dsqrt(ux * ux + uy * uy);
}

template <class S>
S brightness_t(const S& x, const S& u1) {
  const S I0 = S(3.0) / (S(kPi) * (S(3.0) - u1));
  S c = S(1.0) - x * x;
  if (val(c) < 0.0) c = S(0.0);
  return I0 * (S(1.0) - u1 * (S(1.0) - dsqrt(c)));
}

// f(delta) with its branch fixed: 0 uniform, 1 square-root branch, 2 linear branch
template <class S>
S edge_factor_fixed(const S& delta, int branch) {
  if (branch == 0) return delta + S(0.5);
  if (branch == 1) return (S(0.5) + delta) * S(2.0 / 3.0) * dsqrt(S(1.0) + S(1.0) / (S(2.0) * delta));
  return S(2.0 / 3.0) * delta + S(0.5);
}
int edge_branch(double delta, double u1, double delta_c) {
  if (u1 == 0.0) return 0;
  return (delta >= delta_c && delta > 0.0) ? 1 : 2;
}

// Crossing on a frozen stencil.  Recording: bisection on values (as the primal), tangent by
// implicit differentiation.  Frozen (t_ref given): the same interpolant solved by Newton from
// the reference crossing without bracketing -- the smooth continuation of the reference
// root when the perturbed values no longer bracket rho.
template <class S>
S crossing_t_frozen(const S d[4], int cubic, const S& rho, const double* t_ref) {
  double dv[4] = {val(d[0]), val(d[1]), val(d[2]), val(d[3])};
  double t;
  if (!t_ref) {
    t = crossing_t(dv, cubic, val(rho));
  } else if (!cubic) {
    t = (val(rho) - dv[1]) / (dv[2] - dv[1]);
  } else {
    t = *t_ref;
    for (int it = 0; it < 50; ++it) {
      const double g = lagrange4(dv, t) - val(rho);
      const double h = 1e-7;
      const double dg = (lagrange4(dv, t + h) - lagrange4(dv, t - h)) / (2.0 * h);
      const double step = g / dg;
      t -= step;
      if (std::abs(step) < 1e-15) break;
    }
  }
  if constexpr (std::is_same<S, double>::value) {
    return t;
  } else {
    double l[4], dl[4];
    if (cubic) {
      const double tm1 = t + 1.0, t0 = t, t1 = t - 1.0, t2 = t - 2.0;
      l[0] = -(t0 * t1 * t2) / 6.0;
      l[1] = tm1 * t1 * t2 / 2.0;
      l[2] = -(tm1 * t0 * t2) / 2.0;
      l[3] = tm1 * t0 * t1 / 6.0;
      dl[0] = -(t1 * t2 + t0 * t2 + t0 * t1) / 6.0;
      dl[1] = (t1 * t2 + tm1 * t2 + tm1 * t1) / 2.0;
      dl[2] = -(t0 * t2 + tm1 * t2 + tm1 * t0) / 2.0;
      dl[3] = (t0 * t1 + tm1 * t1 + tm1 * t0) / 6.0;
    } else {
      l[0] = 0.0;
      l[1] = 1.0 - t;
      l[2] = t;
      l[3] = 0.0;
      dl[0] = 0.0;
      dl[1] = -1.0;
      dl[2] = 1.0;
      dl[3] = 0.0;
    }
    double Lp = 0.0;
    for (int j = 0; j < 4; ++j) Lp += dl[j] * dv[j];
    S r(t);
    for (int k = 0; k < kNT; ++k) {
      double num = rho.d[k];
      for (int j = 0; j < 4; ++j) num -= l[j] * d[j].d[k];
      r.d[k] = num / Lp;
    }
    return r;
  }
}

// Decisions of one sector: chi per node, the edge-factor branch and the crossing per
// (node, side).
struct Pattern {
  std::vector<char> chi;     // [nr][nth]
  std::vector<char> branch;  // [nr][nth][2]
  std::vector<double> tref;  // [nr][nth][2]
};

// Flux of one sector in scalar type S.  With record != nullptr the decisions are taken
// from the values computed here and stored; otherwise they are read from *frozen.
template <class S>
S sector_flux_t(const LensT<S>& L, const S& wx, const S& wy, const S& rho, const S& u1, double delta_c, int nr,
                int nth, const Sector& Sc, Pattern* record, const Pattern* frozen) {
  const double dr = (Sc.r_hi - Sc.r_lo) / nr;
  const double dth = (Sc.th_hi - Sc.th_lo) / nth;
  if (record) {
    record->chi.assign((size_t)nr * nth, 0);
    record->branch.assign((size_t)nr * nth * 2, 0);
    record->tref.assign((size_t)nr * nth * 2, 0.0);
  }
  std::vector<S> d(nth);
  S total(0.0);
  for (int i = 0; i < nr; ++i) {
    const double ri = Sc.r_lo + (i + 0.5) * dr;
    for (int l = 0; l < nth; ++l) {
      const double th = Sc.th_lo + (l + 0.5) * dth;
      d[l] = node_distance(L, ri * std::cos(th), ri * std::sin(th), wx, wy);
    }
    auto inside = [&](int l) -> bool {
      if (record) {
        const bool in = val(d[l]) < val(rho);
        record->chi[(size_t)i * nth + l] = in;
        return in;
      }
      return frozen->chi[(size_t)i * nth + l] != 0;
    };
    std::vector<char> in(nth);
    for (int l = 0; l < nth; ++l) in[l] = inside(l);
    S row(0.0);
    for (int l = 0; l < nth; ++l) {
      if (!in[l]) continue;
      S W(1.0);
      for (int side = 0; side < 2; ++side) {
        const bool at_edge = !Sc.periodic && (side == 0 ? l == 0 : l == nth - 1);
        int br;
        if (at_edge) {
          br = record ? edge_branch(0.5, val(u1), delta_c) : frozen->branch[((size_t)i * nth + l) * 2 + side];
          if (record) record->branch[((size_t)i * nth + l) * 2 + side] = (char)br;
          W = W + edge_factor_fixed(S(0.5), br) - S(1.0);
          continue;
        }
        const int nb = side == 0 ? (l - 1 + nth) % nth : (l + 1) % nth;
        if (in[nb]) continue;
        const int p = side == 0 ? nb : l;
        S st[4];
        int cubic = 1;
        for (int j = -1; j <= 2; ++j) {
          int idx = p + j;
          if (Sc.periodic) {
            idx = (idx % nth + nth) % nth;
          } else if (idx < 0 || idx >= nth) {
            cubic = 0;
            idx = std::min(std::max(idx, 0), nth - 1);
          }
          st[j + 1] = d[idx];
        }
        const size_t slot = ((size_t)i * nth + l) * 2 + side;
        const S t = crossing_t_frozen(st, cubic, rho, record ? nullptr : &frozen->tref[slot]);
        if (record) record->tref[slot] = val(t);
        const S delta = side == 0 ? S(1.0) - t : t;
        br = record ? edge_branch(val(delta), val(u1), delta_c) : frozen->branch[((size_t)i * nth + l) * 2 + side];
        if (record) record->branch[((size_t)i * nth + l) * 2 + side] = (char)br;
        W = W + edge_factor_fixed(delta, br) - S(1.0);
      }
      row = row + brightness_t(d[l] / rho, u1) * W;
    }
    total = total + S(ri * dth * dr) * row;
  }
  return total;
}

}  // namespace

// =======================================================================================
namespace {

// ---------------------------------------------------------------------------------------
// O14: point-source magnification as a function of the event parameters and its gradient
// through the roots (Sec. 3.5).  The images z* are roots of eq. lens_eq_z, P(z*; b) = 0 with
// coefficients b(params); differentiating that identity gives the paper's root derivative
//   dz*/db_l = -(z*)^l / P'(z*)        (ascending powers: dP/db_l = z^l),
// so with the tangents db/dparams of the coefficients (dual numbers through O4's
// construction) each image moves by dz* = -(sum_l z*^l db_l) / P'(z*).  Eq. amp_point
// then gives A = sum_j 1/|det J(z_j)| with eq. detJ evaluated in dual numbers, through the
// moved images and the parameter-dependent masses and positions.

// Complex dual number: value and eleven tangents in the real and the imaginary part.
struct DC {
  Dual x, y;
};
DC operator+(const DC& a, const DC& b) { return {a.x + b.x, a.y + b.y}; }
DC operator-(const DC& a, const DC& b) { return {a.x - b.x, a.y - b.y}; }
DC operator*(const DC& a, const DC& b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
DC operator/(const DC& a, const DC& b) {
  const Dual n = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / n, (a.y * b.x - a.x * b.y) / n};
}
DC dconj(const DC& a) { return {a.x, -a.y}; }
DC dc(const Dual& x) { return {x, Dual(0.0)}; }

// Polynomials with dual-number coefficients (O4's factors in dual arithmetic).
using PolyD = std::vector<DC>;
PolyD dpmul(const PolyD& a, const PolyD& b) {
  PolyD c(a.size() + b.size() - 1, dc(Dual(0.0)));
  for (size_t i = 0; i < a.size(); ++i)
    for (size_t j = 0; j < b.size(); ++j) c[i + j] = c[i + j] + a[i] * b[j];
  return c;
}
PolyD dpadd(const PolyD& a, const PolyD& b) {
  PolyD c(std::max(a.size(), b.size()), dc(Dual(0.0)));
  for (size_t i = 0; i < a.size(); ++i) c[i] = c[i] + a[i];
  for (size_t i = 0; i < b.size(); ++i) c[i] = c[i] + b[i];
  return c;
}
PolyD dpscale(const PolyD& a, const DC& s) {
  PolyD c(a);
  for (auto& x : c) x = x * s;
  return c;
}
// Value and z-derivative of a polynomial (ascending coefficients) at z, by Horner.
void horner_vd(const PolyD& c, const DC& z, DC* v, DC* d) {
  DC val = c.back(), der = dc(Dual(0.0));
  for (int j = static_cast<int>(c.size()) - 2; j >= 0; --j) {
    der = der * z + val;
    val = val * z + c[j];
  }
  *v = val;
  *d = der;
}

// A_ps at the source centre of epoch t and dA_ps/dparams (11 entries; rho and u1 do not
// enter).  Returns the image-finding status bits.  The root derivative needs
// sum_l z*^l db_l = dP/dparams at fixed z and P'(z*).  Both are evaluated at the root
// through O4's factors rather than through the expanded coefficients: the expanded sum
// cancels to a small fraction of its terms at clustered roots (a low-mass companion),
// while each factor (degree <= N) keeps its own rounding small.
//   P = (z - w) prod_i D_i - H sum_i eps_i prod_{j != i} D_j
uint32_t point_mag_jacobian(int n_lens, const double* p, double t, double* A_out, double* jac) {
  const Lens L = make_lens(n_lens, p);
  const cplx wc = source_center(p, t);
  std::vector<cplx> img;
  const uint32_t st = find_images(L, wc, img);
  Dual pd[kNT];
  for (int k = 0; k < kNT; ++k) {
    pd[k] = Dual(p[k]);
    pd[k].d[k] = 1.0;
  }
  const LensT<Dual> Ld = make_lens_t<Dual>(n_lens, pd);
  DC w;
  source_center_t<Dual>(pd, t, &w.x, &w.y);
  const int n = Ld.n;
  const DC one = dc(Dual(1.0)), zero = dc(Dual(0.0));
  std::vector<DC> a(n);
  for (int k = 0; k < n; ++k) a[k] = {Ld.ax[k], Ld.ay[k]};
  PolyD H{one};
  for (int k = 0; k < n; ++k) H = dpmul(H, PolyD{zero - a[k], one});
  PolyD G = dpscale(H, dconj(w));
  for (int k = 0; k < n; ++k) {
    PolyD Pk{one};
    for (int j = 0; j < n; ++j)
      if (j != k) Pk = dpmul(Pk, PolyD{zero - a[j], one});
    G = dpadd(G, dpscale(Pk, dc(Ld.eps[k])));
  }
  std::vector<PolyD> D(n);
  for (int i = 0; i < n; ++i) D[i] = dpadd(G, dpscale(H, zero - dconj(a[i])));
  Dual A(0.0);
  for (const cplx& z : img) {
    const DC zz{Dual(z.real()), Dual(z.imag())};
    DC Hv, Hd;
    horner_vd(H, zz, &Hv, &Hd);
    std::vector<DC> Dv(n), Dd(n);
    for (int i = 0; i < n; ++i) horner_vd(D[i], zz, &Dv[i], &Dd[i]);
    // P(z) and P'(z) by the product rule on the factors
    DC prodD = one, dprodD = zero;
    for (int i = 0; i < n; ++i) {
      dprodD = dprodD * Dv[i] + prodD * Dd[i];
      prodD = prodD * Dv[i];
    }
    DC S = zero, dS = zero;  // sum_i eps_i prod_{j != i} D_j and its z-derivative
    for (int i = 0; i < n; ++i) {
      DC q = dc(Ld.eps[i]), dq = zero;
      for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        dq = dq * Dv[j] + q * Dd[j];
        q = q * Dv[j];
      }
      S = S + q;
      dS = dS + dq;
    }
    const DC Pz = (zz - w) * prodD - Hv * S;                      // tangents: dP/dparams at z
    const DC Pp = prodD + (zz - w) * dprodD - Hd * S - Hv * dS;   // value: P'(z)
    const cplx dP(Pp.x.v, Pp.y.v);
    DC zd{Dual(z.real()), Dual(z.imag())};
    for (int k = 0; k < kNT; ++k) {
      const cplx dz = -cplx(Pz.x.d[k], Pz.y.d[k]) / dP;  // dz*/db . db/dparams (Sec. 3.5)
      zd.x.d[k] = dz.real();
      zd.y.d[k] = dz.imag();
    }
    // eq. detJ: det J = 1 - |sum_i eps_i / (conj(z) - conj(a_i))^2|^2
    DC kap = zero;
    for (int i = 0; i < Ld.n; ++i) {
      const DC d = dconj(zd - DC{Ld.ax[i], Ld.ay[i]});
      kap = kap + dc(Ld.eps[i]) / (d * d);
    }
    const Dual det = Dual(1.0) - (kap.x * kap.x + kap.y * kap.y);
    A = A + (det.v > 0.0 ? Dual(1.0) / det : Dual(-1.0) / det);
  }
  *A_out = A.v;
  for (int k = 0; k < kNT; ++k) jac[k] = A.d[k];
  return st;
}

// ---------------------------------------------------------------------------------------
// O15: which epochs need the extended-source computation (Sec. 3.4, item iii: only a
// preselected set of N_ext epochs, e.g. near caustics, is modelled with finite-source
// effects; the paper gives no selection rule).  Reading: n_check points on the circle of
// radius guard x rho around the source centre are solved like the centre; the epoch is
// extended when (1) any of them has a different image count or a root/validation flag (a
// caustic crosses the circle), (2) the mean of their point-source magnifications differs from
// the centre's by more than tol A_ps (that mean minus A_ps measures the Laplacian of A_ps,
// the leading finite-source term), or (3) any one differs by more than vary_max A_ps (a
// low-order expansion does not hold).  Every other epoch takes A_ps of eq. amp_point.
constexpr uint32_t ST_POINT = 2048u;  // the epoch took the point-source magnification

bool needs_extended(const Lens& L, const double* p, double t, int n_check, double guard, double tol,
                    double vary_max, double* A_centre) {
  const cplx wc = source_center(p, t);
  std::vector<cplx> img;
  const uint32_t st = find_images(L, wc, img);
  double Ac = 0.0;
  for (const cplx& z : img) Ac += 1.0 / std::abs(1.0 - std::norm(kappa_of(L, z)));
  *A_centre = Ac;
  if (st) return true;
  const double rad = guard * p[6];
  double sum = 0.0, worst = 0.0;
  for (int k = 0; k < n_check; ++k) {
    const double ang = 2.0 * kPi * k / n_check;
    const cplx w = wc + rad * cplx(std::cos(ang), std::sin(ang));
    std::vector<cplx> ik;
    if (find_images(L, w, ik) || ik.size() != img.size()) return true;
    double Ak = 0.0;
    for (const cplx& z : ik) Ak += 1.0 / std::abs(1.0 - std::norm(kappa_of(L, z)));
    sum += Ak;
    worst = std::max(worst, std::abs(Ak - Ac));
  }
  if (std::abs(sum / n_check - Ac) > tol * Ac) return true;
  if (worst > vary_max * Ac) return true;
  return false;
}

}  // namespace

// C entry points for ctypes (tests only).  Complex numbers are passed as (re, im) pairs.
extern "C" {

int orc_abi_version() { return 1; }

// Threads an OpenMP parallel region of the oracle will use.
int orc_num_threads() {
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
}

// Sets the thread count of the oracle's later parallel regions (n >= 1).
void orc_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

void orc_frame(int n_lens, const double* params, double* eps, double* a) {
  const Lens L = make_lens(n_lens, params);
  for (int i = 0; i < n_lens; ++i) {
    eps[i] = L.eps[i];
    a[2 * i] = L.a[i].real();
    a[2 * i + 1] = L.a[i].imag();
  }
}

void orc_source_center(const double* params, double t, double* wc) {
  const cplx w = source_center(params, t);
  wc[0] = w.real();
  wc[1] = w.imag();
}

// Lens given directly by masses and positions (n <= 3).
static Lens lens_from(int n, const double* eps, const double* a) {
  Lens L;
  L.n = n;
  for (int i = 0; i < n; ++i) {
    L.eps[i] = eps[i];
    L.a[i] = cplx(a[2 * i], a[2 * i + 1]);
  }
  return L;
}

void orc_lens_map(int n, const double* eps, const double* a, const double* z, double* w) {
  const cplx r = lens_map(lens_from(n, eps, a), cplx(z[0], z[1]));
  w[0] = r.real();
  w[1] = r.imag();
}

int orc_lens_poly(int n, const double* eps, const double* a, const double* w, double* coef) {
  const Poly P = lens_polynomial(lens_from(n, eps, a), cplx(w[0], w[1]));
  for (size_t j = 0; j < P.size(); ++j) {
    coef[2 * j] = P[j].real();
    coef[2 * j + 1] = P[j].imag();
  }
  return static_cast<int>(P.size()) - 1;
}

int orc_ea_roots(int deg, const double* coef, double* roots, int* iters) {
  Poly P(deg + 1);
  for (int j = 0; j <= deg; ++j) P[j] = cplx(coef[2 * j], coef[2 * j + 1]);
  std::vector<cplx> z;
  const bool ok = ea_roots(P, z, iters);
  for (int k = 0; k < deg; ++k) {
    roots[2 * k] = z[k].real();
    roots[2 * k + 1] = z[k].imag();
  }
  return ok ? 1 : 0;
}

// Ehrlich-Aberth continued from the estimates in roots (in/out) with the step test only, at
// most cap iterations (the validation's last resort); returns 1 when every root converged.
int orc_ea_continue(int deg, const double* coef, double* roots, int cap) {
  Poly P(deg + 1);
  for (int j = 0; j <= deg; ++j) P[j] = cplx(coef[2 * j], coef[2 * j + 1]);
  std::vector<cplx> z(deg);
  for (int k = 0; k < deg; ++k) z[k] = cplx(roots[2 * k], roots[2 * k + 1]);
  int it = 0;
  const bool ok = ea_roots(P, z, &it, true, cap);
  for (int k = 0; k < deg; ++k) {
    roots[2 * k] = z[k].real();
    roots[2 * k + 1] = z[k].imag();
  }
  return ok ? 1 : 0;
}

// Newton polish of one candidate z on the lens equation (the validation's step rule);
// returns |F| at the result.
double orc_polish(int n, const double* eps, const double* a, const double* w, double* z) {
  const Lens L = lens_from(n, eps, a);
  const cplx ww(w[0], w[1]);
  const cplx r = polish(L, ww, cplx(z[0], z[1]));
  z[0] = r.real();
  z[1] = r.imag();
  return std::abs(lens_map(L, r) - ww);
}

// Validated images of a point source at w; returns the count, status bits in *status.
int orc_images(int n, const double* eps, const double* a, const double* w, double* z, uint32_t* status) {
  std::vector<cplx> img;
  const uint32_t st = find_images(lens_from(n, eps, a), cplx(w[0], w[1]), img);
  for (size_t j = 0; j < img.size(); ++j) {
    z[2 * j] = img[j].real();
    z[2 * j + 1] = img[j].imag();
  }
  if (status) *status = st;
  return static_cast<int>(img.size());
}

// eq. amp_point: A = sum_j 1/|det J(z_j)|; parities (sign det J) and per-image |mu| returned.
double orc_point_mag(int n, const double* eps, const double* a, const double* w, int* n_img, double* mu_signed) {
  const Lens L = lens_from(n, eps, a);
  std::vector<cplx> img;
  find_images(L, cplx(w[0], w[1]), img);
  double A = 0.0;
  for (size_t j = 0; j < img.size(); ++j) {
    const double det = 1.0 - std::norm(kappa_of(L, img[j]));
    A += 1.0 / std::abs(det);
    if (mu_signed) mu_signed[j] = 1.0 / det;
  }
  if (n_img) *n_img = static_cast<int>(img.size());
  return A;
}

double orc_brightness(double x, double u1) { return brightness(x, u1); }
double orc_edge_factor(double delta, double u1, double delta_c) { return edge_factor(delta, u1, delta_c); }
double orc_crossing_t(const double* d4, int cubic, double rho) { return crossing_t(d4, cubic, rho); }

// Sectors from given image-limb points (r, theta); returns the count (<= cap).
int orc_build_sectors(int n_pts, const double* r, const double* th, double rho, int cap, double* sec, int* periodic,
                      uint32_t* status) {
  std::vector<double> rr(r, r + n_pts), tt(th, th + n_pts);
  std::vector<Sector> S;
  const uint32_t st = build_sectors(rr, tt, rho, cap, S);
  for (size_t s = 0; s < S.size(); ++s) {
    sec[4 * s + 0] = S[s].r_lo;
    sec[4 * s + 1] = S[s].r_hi;
    sec[4 * s + 2] = S[s].th_lo;
    sec[4 * s + 3] = S[s].th_hi;
    periodic[s] = S[s].periodic ? 1 : 0;
  }
  if (status) *status = st;
  return static_cast<int>(S.size());
}

// O12 retry step on a given list: sec [n][4], periodic [n], clip bits [n] (1 first row,
// 2 last row, 4 first column, 8 last column); writes the new list and returns its length.
int orc_retry_sectors(int n, const double* sec, const int* periodic, const int* clips, double* out, int* out_per) {
  std::vector<Sector> S(n);
  std::vector<int> c(clips, clips + n);
  for (int i = 0; i < n; ++i) S[i] = Sector{sec[4 * i], sec[4 * i + 1], sec[4 * i + 2], sec[4 * i + 3], periodic[i] != 0};
  retry_sectors(S, c);
  for (size_t i = 0; i < S.size(); ++i) {
    out[4 * i + 0] = S[i].r_lo;
    out[4 * i + 1] = S[i].r_hi;
    out[4 * i + 2] = S[i].th_lo;
    out[4 * i + 3] = S[i].th_hi;
    out_per[i] = S[i].periodic ? 1 : 0;
  }
  return static_cast<int>(S.size());
}

// Quadrature over one given sector (no retries).  Returns the un-normalised flux
// (divide by rho^2 for the sector's magnification share).
double orc_sector_flux(int n, const double* eps, const double* a, const double* wc, double rho, double u1,
                       double delta_c, int nr, int nth, const double* sec4, int periodic, int* clip) {
  const Lens L = lens_from(n, eps, a);
  Sector S{sec4[0], sec4[1], sec4[2], sec4[3], periodic != 0};
  return sector_flux(L, cplx(wc[0], wc[1]), rho, u1, delta_c, nr, nth, S, clip);
}

// Whole light curve for one event.  params: [s, q, u0, alpha, t0, tE, rho, u1, q3, r3, psi].
// sec_out: [n_epochs][kmax][4] (r_lo, r_hi, th_lo, th_hi), periodic_out [n_epochs][kmax],
// nsec_out [n_epochs]; any of these may be NULL.  a_ps_out [n_epochs] may be NULL.
void orc_magnification(int n_lens, const double* params, int64_t n_epochs, const double* t, int n_limb, int n_r,
                       int n_theta, double delta_c, int max_retries, int kmax, double* mag, uint32_t* status,
                       double* sec_out, uint8_t* periodic_out, int32_t* nsec_out, double* a_ps_out) {
  const Lens L = make_lens(n_lens, params);
  const Config cfg{n_limb, n_r, n_theta, max_retries, delta_c};
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n_epochs; ++e) {
    std::vector<Sector> S;
    uint32_t st = 0;
    double aps = 0.0;
    mag[e] = epoch_magnification(L, params, t[e], cfg, &st, S, &aps, nullptr);
    status[e] = st;
    if (a_ps_out) a_ps_out[e] = aps;
    if (nsec_out) nsec_out[e] = static_cast<int32_t>(S.size());
    for (size_t s = 0; s < S.size() && static_cast<int>(s) < kmax; ++s) {
      if (sec_out) {
        double* o = sec_out + (e * kmax + s) * 4;
        o[0] = S[s].r_lo;
        o[1] = S[s].r_hi;
        o[2] = S[s].th_lo;
        o[3] = S[s].th_hi;
      }
      if (periodic_out) periodic_out[e * kmax + s] = S[s].periodic ? 1 : 0;
    }
  }
}

// Same quadrature on caller-given sectors (one pass, no retries): the "given grid" mode.
void orc_magnification_given(int n_lens, const double* params, int64_t n_epochs, const double* t, int n_r,
                             int n_theta, double delta_c, int kmax, const double* sec, const uint8_t* periodic,
                             const int32_t* nsec, double* mag, uint32_t* status) {
  const Lens L = make_lens(n_lens, params);
  const double rho = params[6], u1 = params[7];
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n_epochs; ++e) {
    const cplx wc = source_center(params, t[e]);
    double flux = 0.0;
    uint32_t st = ST_GIVEN;
    for (int s = 0; s < nsec[e]; ++s) {
      const double* g = sec + (e * kmax + s) * 4;
      Sector S{g[0], g[1], g[2], g[3], periodic[e * kmax + s] != 0};
      int clip = 0;
      flux += sector_flux(L, wc, rho, u1, delta_c, n_r, n_theta, S, &clip);
      if (clip) st |= ST_CLIP;
    }
    mag[e] = flux / (rho * rho);
    if (!std::isfinite(mag[e])) st |= ST_NAN;
    status[e] = st;
  }
}

// Jacobian d mag / d params (all 11 entries; unused ones are 0) on caller-given sectors,
// with the decisions of the evaluation at params itself (forward-mode dual numbers).
void orc_jacobian_given(int n_lens, const double* params, int64_t n_epochs, const double* t, int n_r, int n_theta,
                        double delta_c, int kmax, const double* sec, const uint8_t* periodic, const int32_t* nsec,
                        double* mag, double* jac) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n_epochs; ++e) {
    Dual p[kNT];
    for (int k = 0; k < kNT; ++k) {
      p[k] = Dual(params[k]);
      p[k].d[k] = 1.0;
    }
    const LensT<Dual> L = make_lens_t(n_lens, p);
    Dual wx, wy;
    source_center_t(p, t[e], &wx, &wy);
    Dual flux(0.0);
    for (int s = 0; s < nsec[e]; ++s) {
      const double* g = sec + (e * kmax + s) * 4;
      Sector S{g[0], g[1], g[2], g[3], periodic[e * kmax + s] != 0};
      Pattern pat;
      flux = flux + sector_flux_t(L, wx, wy, p[6], p[7], delta_c, n_r, n_theta, S, &pat, nullptr);
    }
    const Dual m = flux / (p[6] * p[6]);
    mag[e] = m.v;
    for (int k = 0; k < kNT; ++k) jac[e * kNT + k] = m.d[k];
  }
}

// Magnification at params_eval with every decision taken from params_ref (frozen
// structure), on caller-given sectors: the function whose central differences check the
// Jacobian.
void orc_magnification_frozen(int n_lens, const double* params_eval, const double* params_ref, int64_t n_epochs,
                              const double* t, int n_r, int n_theta, double delta_c, int kmax, const double* sec,
                              const uint8_t* periodic, const int32_t* nsec, double* mag) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n_epochs; ++e) {
    const LensT<double> Lr = make_lens_t(n_lens, params_ref);
    const LensT<double> Le = make_lens_t(n_lens, params_eval);
    double wxr, wyr, wxe, wye;
    source_center_t(params_ref, t[e], &wxr, &wyr);
    source_center_t(params_eval, t[e], &wxe, &wye);
    double flux = 0.0;
    for (int s = 0; s < nsec[e]; ++s) {
      const double* g = sec + (e * kmax + s) * 4;
      Sector S{g[0], g[1], g[2], g[3], periodic[e * kmax + s] != 0};
      Pattern pat;
      sector_flux_t(Lr, wxr, wyr, params_ref[6], params_ref[7], delta_c, n_r, n_theta, S, &pat, nullptr);
      flux += sector_flux_t(Le, wxe, wye, params_eval[6], params_eval[7], delta_c, n_r, n_theta, S, nullptr, &pat);
    }
    mag[e] = flux / (params_eval[6] * params_eval[6]);
  }
}

// Finite-source magnification straight from its definition (Sec. 2.2): the brightness-
// weighted mean of the point-source magnification (eq. amp_point) over the source disk.
// Radial nodes: Gauss-Legendre in x on [0, pi/2] with r = sin x (this makes the limb-
// darkening square root sqrt(1 - r^2) = cos x smooth); angular nodes: the trapezoid rule
// (exponentially convergent for a smooth periodic integrand).  Valid only where no caustic
// crosses the disk; count_changes[e] counts disk nodes whose image count differs from the
// centre's (0 means the integrand is smooth).  A reference with no image-plane grid at all.
void orc_disk_mag(int n_lens, const double* params, int64_t n_epochs, const double* t, int n_x, int n_phi,
                  double* mag, int32_t* count_changes) {
  // Gauss-Legendre nodes/weights on [-1, 1] by Newton's method on P_n
  std::vector<double> xs(n_x), ws(n_x);
  for (int i = 0; i < n_x; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (n_x + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n_x; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = n_x == 1 ? x : p1;
      const double pm = n_x == 1 ? 1.0 : p0;
      dp = n_x * (x * pn - pm) / (x * x - 1.0);
      const double dx = pn / dp;
      x -= dx;
      if (std::abs(dx) < 1e-16) break;
    }
    xs[i] = x;
    ws[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  const Lens L = make_lens(n_lens, params);
  const double rho = params[6], u1 = params[7];
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n_epochs; ++e) {
    const cplx wc = source_center(params, t[e]);
    std::vector<cplx> img;
    find_images(L, wc, img);
    const size_t nc = img.size();
    double num = 0.0, den = 0.0;
    int changes = 0;
    for (int i = 0; i < n_x; ++i) {
      const double xx = 0.25 * kPi * (xs[i] + 1.0);  // [0, pi/2]
      const double r = std::sin(xx);
      const double wr = ws[i] * 0.25 * kPi * r * std::cos(xx) * brightness(r, u1);
      for (int j = 0; j < n_phi; ++j) {
        const double ph = 2.0 * kPi * (j + 0.5) / n_phi;
        const cplx w = wc + rho * r * cplx(std::cos(ph), std::sin(ph));
        find_images(L, w, img);
        if (img.size() != nc) ++changes;
        double A = 0.0;
        for (const cplx& z : img) A += 1.0 / std::abs(1.0 - std::norm(kappa_of(L, z)));
        num += wr * A;
        den += wr;
      }
    }
    mag[e] = num / den;
    if (count_changes) count_changes[e] = changes;
  }
}

// O14 for a light curve: a_ps [n_epochs], jac [n_epochs][11] = dA_ps/dparams (through the
// roots, Sec. 3.5), status [n_epochs] (image-finding bits).
void orc_point_jacobian(int n_lens, const double* params, int64_t n_epochs, const double* t, double* a_ps,
                        double* jac, uint32_t* status) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n_epochs; ++e) {
    const uint32_t st = point_mag_jacobian(n_lens, params, t[e], &a_ps[e], jac + e * kNT);
    if (status) status[e] = st;
  }
}

// O15 for a light curve: extended[e] = 1 for epochs that need the finite-source computation;
// a_ps [n_epochs] the centre's point-source magnification.
void orc_hybrid_select(int n_lens, const double* params, int64_t n_epochs, const double* t, int n_check, double guard,
                       double tol, double vary_max, int32_t* extended, double* a_ps) {
  const Lens L = make_lens(n_lens, params);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n_epochs; ++e) {
    double Ac = 0.0;
    extended[e] = needs_extended(L, params, t[e], n_check, guard, tol, vary_max, &Ac) ? 1 : 0;
    a_ps[e] = Ac;
  }
}

// The hybrid light curve (Sec. 3.4, item iii): extended epochs by the full method (as
// orc_magnification), every other epoch A_ps (status ST_POINT).
void orc_hybrid(int n_lens, const double* params, int64_t n_epochs, const double* t, int n_check, double guard,
                double tol, double vary_max, int n_limb, int n_r, int n_theta, double delta_c, int max_retries,
                double* mag, uint32_t* status) {
  const Lens L = make_lens(n_lens, params);
  const Config cfg{n_limb, n_r, n_theta, max_retries, delta_c};
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n_epochs; ++e) {
    double Ac = 0.0;
    if (needs_extended(L, params, t[e], n_check, guard, tol, vary_max, &Ac)) {
      std::vector<Sector> S;
      uint32_t st = 0;
      double aps = 0.0;
      mag[e] = epoch_magnification(L, params, t[e], cfg, &st, S, &aps, nullptr);
      status[e] = st;
    } else {
      mag[e] = Ac;
      status[e] = ST_POINT;
    }
  }
}

}  // extern "C"
