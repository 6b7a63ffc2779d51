// Float64 operator tables for the FMM (see tables.hpp for the basis).
#include "tables.hpp"

#include <array>
#include <cmath>
#include <mutex>
#include <random>

namespace mahi {

namespace {

constexpr double kPi = 3.14159265358979323846;

// log of s_n^m = sqrt((n+|m|)! (n-|m|)!)
double lsf(int n, int m) {
  m = std::abs(m);
  return 0.5 * (std::lgamma(n + m + 1.0) + std::lgamma(n - m + 1.0));
}

// Schmidt-normalised irregular harmonics It_n^m, m >= 0, n <= P, at index n(n+1)/2 + m,
// from the unnormalised recurrences (I_n^m = (n-m)! P_n^m e^{imf} / r^{n+1}).
void irregular_schmidt(int P, double x, double y, double z, cplx *out) {
  const double r2 = x * x + y * y + z * z;
  const double ir2 = 1.0 / r2;
  std::vector<cplx> I((P + 1) * (P + 2) / 2);
  auto at = [](int n, int m) { return n * (n + 1) / 2 + m; };
  I[0] = cplx(1.0 / std::sqrt(r2), 0.0);
  const cplx xy(x, y);
  for (int m = 1; m <= P; ++m) I[at(m, m)] = -double(2 * m - 1) * xy * ir2 * I[at(m - 1, m - 1)];
  for (int m = 0; m < P; ++m) I[at(m + 1, m)] = double(2 * m + 1) * z * ir2 * I[at(m, m)];
  for (int m = 0; m <= P; ++m)
    for (int n = m + 2; n <= P; ++n)
      I[at(n, m)] = (double(2 * n - 1) * z * I[at(n - 1, m)] - double((n - 1) * (n - 1) - m * m) * I[at(n - 2, m)]) * ir2;
  for (int n = 0; n <= P; ++n)
    for (int m = 0; m <= n; ++m) out[at(n, m)] = I[at(n, m)] * std::exp(-lsf(n, m));
}

// Accessor for any m from a table holding m >= 0.
inline cplx full(const cplx *t, int n, int m) {
  if (m >= 0) return t[n * (n + 1) / 2 + m];
  cplx c = std::conj(t[n * (n + 1) / 2 - m]);
  return (m & 1) ? -c : c;
}

// Assemble the real matrix of the linear map
//   L_k^l (l >= 0) = sum_{n, m=-n..n} G(k,l,n,m) M_n^m ,  M_n^{-m} = (-1)^m conj(M_n^m).
template <class Gf>
void assemble(int p, Gf G, double *T) {
  const int K = ncoef(p);
  for (int i = 0; i < K * K; ++i) T[i] = 0.0;
  for (int k = 0; k <= p; ++k)
    for (int l = 0; l <= k; ++l)
      for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
          const cplx A = G(k, l, n, m);
          const int ra = ridx(k, l, 0), rb = ridx(k, l, 1);
          const int ca = ridx(n, m, 0), cb = ridx(n, m, 1);
          if (m == 0) {
            T[ra * K + ca] += A.real();
            if (l > 0) T[rb * K + ca] += A.imag();
          } else {
            cplx B = G(k, l, n, -m);
            if (m & 1) B = -B;
            const cplx P = A + B, Mi = A - B;
            T[ra * K + ca] += P.real();
            T[ra * K + cb] += -Mi.imag();
            if (l > 0) {
              T[rb * K + ca] += P.imag();
              T[rb * K + cb] += Mi.real();
            }
          }
        }
}

}  // namespace

void regular_schmidt(int p, double x, double y, double z, cplx *out) {
  auto at = [](int n, int m) { return n * (n + 1) / 2 + m; };
  const double r2 = x * x + y * y + z * z;
  out[0] = cplx(1.0, 0.0);
  const cplx xy(x, y);
  for (int m = 1; m <= p; ++m) out[at(m, m)] = -std::sqrt((2.0 * m - 1.0) / (2.0 * m)) * xy * out[at(m - 1, m - 1)];
  for (int m = 0; m < p; ++m) out[at(m + 1, m)] = std::sqrt(2.0 * m + 1.0) * z * out[at(m, m)];
  for (int m = 0; m <= p; ++m)
    for (int n = m + 2; n <= p; ++n)
      out[at(n, m)] = (double(2 * n - 1) * z * out[at(n - 1, m)] -
                       std::sqrt(double((n - 1) * (n - 1) - m * m)) * r2 * out[at(n - 2, m)]) /
                      std::sqrt(double(n * n - m * m));
}

void m2m_matrix(int p, const double d[3], double *T) {
  std::vector<cplx> R((p + 1) * (p + 2) / 2);
  regular_schmidt(p, d[0], d[1], d[2], R.data());
  // Mt'_n^m = sum_{k,l} 2^-k s_n^m / (s_k^l s_{n-k}^{m-l}) conj(Rt_{n-k}^{m-l}(d)) Mt_k^l
  assemble(p, [&](int n, int m, int k, int l) -> cplx {
    if (k > n || std::abs(m - l) > n - k) return cplx(0, 0);
    const double f = std::ldexp(std::exp(lsf(n, m) - lsf(k, l) - lsf(n - k, m - l)), -k);
    return f * std::conj(full(R.data(), n - k, m - l));
  }, T);
}

void l2l_matrix(int p, const double d[3], double *T) {
  std::vector<cplx> R((p + 1) * (p + 2) / 2);
  regular_schmidt(p, d[0], d[1], d[2], R.data());
  // Lt^c_a^b = 2^{-a-1} sum_{k,l} s_k^l / (s_a^b s_{k-a}^{l-b}) conj(Rt_{k-a}^{l-b}(d)) Lt_k^l
  assemble(p, [&](int a, int b, int k, int l) -> cplx {
    if (k < a || std::abs(l - b) > k - a) return cplx(0, 0);
    const double f = std::ldexp(std::exp(lsf(k, l) - lsf(a, b) - lsf(k - a, l - b)), -a - 1);
    return f * std::conj(full(R.data(), k - a, l - b));
  }, T);
}

void m2l_matrix(int p, const double v[3], double *T) {
  std::vector<cplx> I((2 * p + 1) * (2 * p + 2) / 2);
  irregular_schmidt(2 * p, v[0], v[1], v[2], I.data());
  // Lt_k^l = (-1)^k sum_{n,m} s_{n+k}^{m+l} / (s_k^l s_n^m) It_{n+k}^{m+l}(v) Mt_n^m
  assemble(p, [&](int k, int l, int n, int m) -> cplx {
    const double f = std::exp(lsf(n + k, m + l) - lsf(k, l) - lsf(n, m));
    const cplx c = f * full(I.data(), n + k, m + l);
    return (k & 1) ? -c : c;
  }, T);
}

double ewald_unit_cube(const double r[3]) {
  // phi_EW for a unit cube: real-space erfc sum + reciprocal sum - pi/alpha^2.
  const double alpha = 2.0;
  double rr[3];
  for (int d = 0; d < 3; ++d) rr[d] = r[d] - std::floor(r[d] + 0.5);
  const bool zero = rr[0] == 0 && rr[1] == 0 && rr[2] == 0;
  double s = 0.0;
  const int R = 5;
  for (int a = -R; a <= R; ++a)
    for (int b = -R; b <= R; ++b)
      for (int c = -R; c <= R; ++c) {
        if (zero && a == 0 && b == 0 && c == 0) continue;
        const double x = rr[0] + a, y = rr[1] + b, z = rr[2] + c;
        const double d = std::sqrt(x * x + y * y + z * z);
        if (d > 9.0) continue;
        s += std::erfc(alpha * d) / d;
      }
  if (zero) s -= 2.0 * alpha / std::sqrt(kPi);
  const int Mx = 6;
  for (int a = 0; a <= Mx; ++a)
    for (int b = -Mx; b <= Mx; ++b)
      for (int c = -Mx; c <= Mx; ++c) {
        if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
        const double k2 = 4 * kPi * kPi * double(a * a + b * b + c * c);
        const double w = 2.0 * 4 * kPi * std::exp(-k2 / (4 * alpha * alpha)) / k2;
        s += w * std::cos(2 * kPi * (a * rr[0] + b * rr[1] + c * rr[2]));
      }
  return s - kPi / (alpha * alpha);
}

const std::vector<cplx> &lattice_coefficients(int jmax) {
  static std::mutex mu;
  static std::vector<cplx> cache;
  static int cached = -1;
  std::lock_guard<std::mutex> lock(mu);
  if (cached >= jmax) return cache;
  // Project h on a sphere of radius rho with Gauss-Legendre nodes in cos(theta)
  // and uniform nodes in phi:  Ht_j^m = (2j+1)/(4 pi rho^j) int h(rho s) Rt_j^m(s) dOmega.
  const double rho = 1.2;
  const int nth = std::max(64, jmax + 48), nph = 2 * nth;
  std::vector<double> xg(nth), wg(nth);
  for (int i = 0; i < nth; ++i) {  // Gauss-Legendre nodes by Newton iteration
    double x = std::cos(kPi * (i + 0.75) / (nth + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= nth; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = nth * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= nth; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double dp = nth * (x * p1 - p0) / (x * x - 1.0);
    xg[i] = x;
    wg[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  const int nj = (jmax + 1) * (jmax + 2) / 2;
  std::vector<cplx> acc(nj, cplx(0, 0)), R(nj);
  for (int i = 0; i < nth; ++i) {
    const double ct = xg[i], st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
    for (int k = 0; k < nph; ++k) {
      const double ph = 2 * kPi * k / nph;
      const double s[3] = {st * std::cos(ph), st * std::sin(ph), ct};
      const double r[3] = {rho * s[0], rho * s[1], rho * s[2]};
      double near = 0.0;
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
          for (int c = -1; c <= 1; ++c) {
            const double x = r[0] + a, y = r[1] + b, z = r[2] + c;
            near += 1.0 / std::sqrt(x * x + y * y + z * z);
          }
      const double h = ewald_unit_cube(r) - near - (2 * kPi / 3.0) * rho * rho;
      regular_schmidt(jmax, s[0], s[1], s[2], R.data());
      const double w = wg[i] * 2 * kPi / nph * h;
      for (int t = 0; t < nj; ++t) acc[t] += w * R[t];
    }
  }
  cache.assign(nj, cplx(0, 0));
  for (int j = 0; j <= jmax; ++j)
    for (int m = 0; m <= j; ++m) {
      const int t = j * (j + 1) / 2 + m;
      cache[t] = (2.0 * j + 1.0) / (4 * kPi * std::pow(rho, j)) * acc[t];
    }
  cached = jmax;
  return cache;
}

void lattice_matrix(int p, double *T) {
  const std::vector<cplx> &H = lattice_coefficients(2 * p);
  // Lt_k^l = sum_{n,b} (-1)^n s_{n+k}^{b+l} / (s_k^l s_n^b) Ht_{n+k}^{b+l} Mt_n^b
  assemble(p, [&](int k, int l, int n, int b) -> cplx {
    if (std::abs(b + l) > n + k) return cplx(0, 0);
    const double f = std::exp(lsf(n + k, b + l) - lsf(k, l) - lsf(n, b));
    const cplx c = f * full(H.data(), n + k, b + l);
    return (n & 1) ? -c : c;
  }, T);
}

namespace {

// phi(c + h u) from a real-packed local expansion (h = 1).
double eval_local(int p, const std::vector<double> &L, const double u[3]) {
  std::vector<cplx> R((p + 1) * (p + 2) / 2);
  regular_schmidt(p, u[0], u[1], u[2], R.data());
  double s = 0.0;
  for (int n = 0; n <= p; ++n) {
    s += L[ridx(n, 0, 0)] * R[n * (n + 1) / 2].real();
    for (int m = 1; m <= n; ++m)
      s += 2.0 * (L[ridx(n, m, 0)] * R[n * (n + 1) / 2 + m].real() + L[ridx(n, m, 1)] * R[n * (n + 1) / 2 + m].imag());
  }
  return s;
}

std::vector<double> p2m(int p, const std::vector<std::array<double, 4>> &pts, double scale, const double c[3]) {
  const int K = ncoef(p);
  std::vector<double> M(K, 0.0);
  std::vector<cplx> R((p + 1) * (p + 2) / 2);
  for (auto &a : pts) {
    regular_schmidt(p, (a[0] - c[0]) / scale, (a[1] - c[1]) / scale, (a[2] - c[2]) / scale, R.data());
    for (int n = 0; n <= p; ++n)
      for (int m = 0; m <= n; ++m) {
        M[ridx(n, m, 0)] += a[3] * R[n * (n + 1) / 2 + m].real();
        if (m) M[ridx(n, m, 1)] -= a[3] * R[n * (n + 1) / 2 + m].imag();
      }
  }
  return M;
}

std::vector<double> matvec(int K, const std::vector<double> &T, const std::vector<double> &x) {
  std::vector<double> y(K, 0.0);
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j) y[i] += T[i * K + j] * x[j];
  return y;
}

}  // namespace

double host_selftest(int p) {
  const int K = ncoef(p);
  std::mt19937_64 rng(17);
  std::uniform_real_distribution<double> U(-0.5, 0.5);
  std::vector<std::array<double, 4>> pts(7);
  for (auto &a : pts) a = {U(rng), U(rng), U(rng), 2 * U(rng)};
  double worst = 0.0;
  std::vector<double> T(K * K);
  // 1) M2M is exact: multipole of a child cloud moved to the parent equals the direct parent multipole.
  {
    const double d[3] = {0.25, -0.25, 0.25}, zero[3] = {0, 0, 0};
    std::vector<std::array<double, 4>> par(pts.size());
    for (size_t i = 0; i < pts.size(); ++i)
      par[i] = {pts[i][0] / 2 + d[0], pts[i][1] / 2 + d[1], pts[i][2] / 2 + d[2], pts[i][3]};
    m2m_matrix(p, d, T.data());
    auto Mc = p2m(p, pts, 1.0, zero), Mp = p2m(p, par, 1.0, zero), Mt = matvec(K, T, Mc);
    double e = 0, nrm = 0;
    for (int i = 0; i < K; ++i) e = std::max(e, std::fabs(Mt[i] - Mp[i])), nrm = std::max(nrm, std::fabs(Mp[i]));
    worst = std::max(worst, e / nrm);
  }
  // 2) M2L then L2L then evaluation against 1/r at a well-separated point (truncation-limited).
  {
    const double v[3] = {4.0, -3.0, 3.0}, zero[3] = {0, 0, 0}, d[3] = {-0.25, 0.25, 0.25};
    m2l_matrix(p, v, T.data());
    auto M = p2m(p, pts, 1.0, zero);
    auto L = matvec(K, T, M);
    std::vector<double> T2(K * K);
    l2l_matrix(p, d, T2.data());
    auto Lc = matvec(K, T2, L);
    const double u[3] = {0.2, -0.1, 0.3};
    const double xp[3] = {v[0] + d[0] + u[0] / 2, v[1] + d[1] + u[1] / 2, v[2] + d[2] + u[2] / 2};
    double ex = 0;
    for (auto &a : pts) ex += a[3] / std::sqrt((xp[0] - a[0]) * (xp[0] - a[0]) + (xp[1] - a[1]) * (xp[1] - a[1]) +
                                               (xp[2] - a[2]) * (xp[2] - a[2]));
    const double got = 2.0 * eval_local(p, Lc, u);  // child box edge is 1/2
    worst = std::max(worst, std::fabs(got - ex) / std::fabs(ex));
  }
  // 3) lattice: truncated bilinear form against psi(a-b) - (2 pi/3)|a-b|^2 on close pairs.
  {
    lattice_matrix(p, T.data());
    const double zero[3] = {0, 0, 0};
    std::vector<std::array<double, 4>> one = {{0.11, -0.07, 0.05, 1.0}};
    auto M = p2m(p, one, 1.0, zero);
    auto L = matvec(K, T, M);
    const double u[3] = {-0.06, 0.09, -0.1};
    const double r[3] = {u[0] - one[0][0], u[1] - one[0][1], u[2] - one[0][2]};
    double near = 0.0;
    for (int a = -1; a <= 1; ++a)
      for (int b = -1; b <= 1; ++b)
        for (int c = -1; c <= 1; ++c) {
          const double x = r[0] + a, y = r[1] + b, z = r[2] + c;
          near += 1.0 / std::sqrt(x * x + y * y + z * z);
        }
    const double h = ewald_unit_cube(r) - near - (2 * kPi / 3.0) * (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double got = eval_local(p, L, u);
    worst = std::max(worst, std::fabs(got - h) / std::fabs(h));
  }
  return worst;
}

}  // namespace mahi
