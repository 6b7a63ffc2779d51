// Host-side float64 generation of the FMM operator tables.
//
// Basis: complex solid harmonics in Schmidt semi-normalised form with the
// Condon-Shortley phase,
//   Rt_n^m(x) = r^n P_n^m(cos t) e^{i m f} sqrt((n-m)!/(n+m)!)        (regular)
//   It_n^m(x) = r^{-n-1} P_n^m(cos t) e^{i m f} sqrt((n-m)!/(n+m)!)   (irregular)
// with Rt_n^{-m} = (-1)^m conj(Rt_n^m).  A multipole about centre c in units of
// the box edge h is Mt_n^m = sum_j q_j conj(Rt_n^m((x_j - c)/h)); a local
// expansion gives phi(c + h u) = (1/h) sum_{n,m} Lt_n^m conj(Rt_n^m(u)).
// Coefficients are stored as (p+1)^2 reals per box: for each degree n the real
// part of m = 0, then (Re, Im) of m = 1..n.  All translation operators act on
// these real vectors as dense (p+1)^2 x (p+1)^2 matrices, built here from the
// addition theorems of the solid harmonics; every table is dimensionless, so
// one table serves all levels of the octree.
#pragma once
#include <complex>
#include <vector>

namespace mahi {

using cplx = std::complex<double>;

inline int ncoef(int p) { return (p + 1) * (p + 1); }
inline int ridx(int n, int m, int im) { return m == 0 ? n * n : n * n + 2 * m - 1 + im; }

// Schmidt-normalised regular harmonics Rt_n^m, m >= 0, at index n(n+1)/2 + m.
void regular_schmidt(int p, double x, double y, double z, cplx *out);

// Real matrices, row-major [rows = ncoef(p)][cols = ncoef(p)].
void m2m_matrix(int p, const double delta[3], double *T);   // child -> parent, delta = (c_child - c_parent)/h_parent
void l2l_matrix(int p, const double delta[3], double *T);   // parent -> child, delta = (c_child - c_parent)/h_parent
void m2l_matrix(int p, const double v[3], double *T);       // source -> target, v = (c_target - c_source)/h
void lattice_matrix(int p, double *T);                      // root multipole -> root local, images with |n|_inf >= 2

// Lattice coefficients Ht_j^m (m >= 0, index j(j+1)/2 + m), j <= jmax, of the
// harmonic part h of the unit-cube lattice remainder
//   psi(r) = phi_Ewald(r) - sum_{|n|_inf <= 1} 1/|r + n| = (2 pi / 3) r^2 + h(r),
// expanded as h(r) = sum_{j,m} Ht_j^m s_j^m conj(R_j^m(r)) (unnormalised R).
const std::vector<cplx> &lattice_coefficients(int jmax);

// Ewald pair kernel of the unit cube (tin-foil, neutralising background);
// used only to build the lattice table and in self-tests.
double ewald_unit_cube(const double r[3]);

// Self-test of the tables against direct sums; returns the largest relative error.
double host_selftest(int p);

}  // namespace mahi
