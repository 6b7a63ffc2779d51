// gfx950 kernels of the MAHI hot path.
//
// One evaluation runs, in order (paper, section "Fast Multipole Method" and
// Fig. fmm_scheme; section "Multipole-Accelerated Hamiltonian Interpolation"):
//   bbox (open boundaries) -> bin -> scan -> scatter -> leaf sort/pack      octree build
//   p2m -> m2m (levels d-1..0) -> lattice                                  upward pass, periodic images
//   m2l (all levels, matrix cores) -> l2l (levels 1..d)                    far field
//   p2p_l2p (near field + far field at the atoms + outputs)                 eq scaled_electrostatics
//   site (per-site correction in float64) -> finalize (energy)             eqs correction_scheme..C_B
// Positions inside the FMM are leaf-local (units of the leaf edge), so the
// float32 path never subtracts large absolute coordinates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "device_common.hpp"
#include "kernels.hpp"

namespace mahi {

// ---------------------------------------------------------------------------
// Recurrence constants of the Schmidt-normalised solid harmonics
// ---------------------------------------------------------------------------
__constant__ double c_sect[kMaxOrder + 2];                   // sqrt((2m-1)/(2m))
__constant__ double c_up[kMaxOrder + 2];                     // sqrt(2m+1)
__constant__ double c_b1[kMaxOrder + 1][kMaxOrder + 1];      // (2n-1)/sqrt(n^2-m^2)
__constant__ double c_b2[kMaxOrder + 1][kMaxOrder + 1];      // sqrt((n-1)^2-m^2)/sqrt(n^2-m^2)
__constant__ double c_dz[kMaxOrder + 1][kMaxOrder + 1];      // sqrt((j+1+b)(j+1-b))
__constant__ double c_r1[kMaxOrder + 1][kMaxOrder + 1];      // sqrt((j+2-b)(j+1-b))
__constant__ double c_r2[kMaxOrder + 1][kMaxOrder + 1];      // sqrt((j+b+2)(j+b+1))

hipError_t upload_constants() {
  double sect[kMaxOrder + 2], up[kMaxOrder + 2];
  static double b1[kMaxOrder + 1][kMaxOrder + 1], b2[kMaxOrder + 1][kMaxOrder + 1];
  static double dz[kMaxOrder + 1][kMaxOrder + 1], r1[kMaxOrder + 1][kMaxOrder + 1], r2[kMaxOrder + 1][kMaxOrder + 1];
  for (int m = 0; m < kMaxOrder + 2; ++m) {
    sect[m] = m > 0 ? sqrt((2.0 * m - 1.0) / (2.0 * m)) : 0.0;
    up[m] = sqrt(2.0 * m + 1.0);
  }
  for (int n = 0; n <= kMaxOrder; ++n)
    for (int m = 0; m <= kMaxOrder; ++m) {
      const double den = double(n * n - m * m);
      b1[n][m] = (m <= n - 2) ? (2.0 * n - 1.0) / sqrt(den) : 0.0;
      b2[n][m] = (m <= n - 2) ? sqrt(double((n - 1) * (n - 1) - m * m)) / sqrt(den) : 0.0;
      dz[n][m] = (m <= n) ? sqrt(double((n + 1 + m) * (n + 1 - m))) : 0.0;
      r1[n][m] = (m <= n) ? sqrt(double((n + 2 - m) * (n + 1 - m))) : 0.0;
      r2[n][m] = (m <= n) ? sqrt(double((n + m + 2) * (n + m + 1))) : 0.0;
    }
  hipError_t e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_sect), sect, sizeof(sect))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_up), up, sizeof(up))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_b1), b1, sizeof(b1))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_b2), b2, sizeof(b2))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_dz), dz, sizeof(dz))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_r1), r1, sizeof(r1))) != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_r2), r2, sizeof(r2));
}

__host__ __device__ inline int ridx_d(int n, int m, int im) { return m == 0 ? n * n : n * n + 2 * m - 1 + im; }

// Visit Rt_n^m(x, y, z) for 0 <= m <= n <= p, m-major, with O(1) registers.
template <class T, class F>
__device__ __forceinline__ void for_regular(int p, T x, T y, T z, F &&f) {
  const T r2 = x * x + y * y + z * z;
  T sr = T(1), si = T(0);
  for (int m = 0; m <= p; ++m) {
    if (m > 0) {
      const T c = -(T)c_sect[m];
      const T nr = c * (x * sr - y * si);
      const T ni = c * (x * si + y * sr);
      sr = nr;
      si = ni;
    }
    f(m, m, sr, si);
    if (m == p) break;
    T r1r = (T)c_up[m] * z * sr, r1i = (T)c_up[m] * z * si;
    f(m + 1, m, r1r, r1i);
    T r0r = sr, r0i = si;
    for (int n = m + 2; n <= p; ++n) {
      const T b1 = (T)c_b1[n][m], b2 = (T)c_b2[n][m];
      const T nr = b1 * z * r1r - b2 * r2 * r0r;
      const T ni = b1 * z * r1i - b2 * r2 * r0i;
      r0r = r1r;
      r0i = r1i;
      r1r = nr;
      r1i = ni;
      f(n, m, nr, ni);
    }
  }
}

// The same recurrence for an order fixed at compile time: the coefficients
// are compile-time constants (tables built by a constexpr constructor) and
// the loops unroll completely, so no coefficient is loaded at run time.
constexpr double csqrt(double x) {  // Newton iteration; compile-time use only
  if (!(x > 0.0)) return 0.0;
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 80; ++i) r = 0.5 * (r + x / r);
  return r;
}

template <int P>
struct RegCoef {
  double sect[P + 2], up[P + 2], b1[P + 1][P + 1], b2[P + 1][P + 1];
  constexpr RegCoef() : sect(), up(), b1(), b2() {
    for (int m = 0; m < P + 2; ++m) {
      sect[m] = m > 0 ? csqrt((2.0 * m - 1.0) / (2.0 * m)) : 0.0;
      up[m] = csqrt(2.0 * m + 1.0);
    }
    for (int n = 0; n <= P; ++n)
      for (int m = 0; m <= P; ++m) {
        const double den = double(n * n - m * m);
        b1[n][m] = (m <= n - 2) ? (2.0 * n - 1.0) / csqrt(den) : 0.0;
        b2[n][m] = (m <= n - 2) ? csqrt(double((n - 1) * (n - 1) - m * m)) / csqrt(den) : 0.0;
      }
  }
};
template <int P>
__device__ constexpr RegCoef<P> kRegCoef{};

template <int P, class T, class F>
__device__ __forceinline__ void for_regular_t(T x, T y, T z, F &&f) {
  const T r2 = x * x + y * y + z * z;
  T sr = T(1), si = T(0);
#pragma unroll
  for (int m = 0; m <= P; ++m) {
    if (m > 0) {
      const T c = -(T)kRegCoef<P>.sect[m];
      const T nr = c * (x * sr - y * si);
      const T ni = c * (x * si + y * sr);
      sr = nr;
      si = ni;
    }
    f(m, m, sr, si);
    if (m < P) {
      T r1r = (T)kRegCoef<P>.up[m] * z * sr, r1i = (T)kRegCoef<P>.up[m] * z * si;
      f(m + 1, m, r1r, r1i);
      T r0r = sr, r0i = si;
#pragma unroll
      for (int n = m + 2; n <= P; ++n) {
        const T b1 = (T)kRegCoef<P>.b1[n][m], b2 = (T)kRegCoef<P>.b2[n][m];
        const T nr = b1 * z * r1r - b2 * r2 * r0r;
        const T ni = b1 * z * r1i - b2 * r2 * r0i;
        r0r = r1r;
        r0i = r1i;
        r1r = nr;
        r1i = ni;
        f(n, m, nr, ni);
      }
    }
  }
}

// Compile-time order PT > 0, else the run-time order p.
template <int PT, class T, class F>
__device__ __forceinline__ void visit_regular(int p, T x, T y, T z, F &&f) {
  if constexpr (PT > 0) for_regular_t<PT>(x, y, z, f);
  else for_regular(p, x, y, z, f);
}

// Derivative local coefficients: for phi = sum L conj(Rt(u)), d phi / du_{x,y,z}
// = sum D_{x,y,z} conj(Rt(u)) over degrees j < p, with each D_j^b formed from
// L_{j+1}^{b-1}, L_{j+1}^b, L_{j+1}^{b+1} (gradient relations of the solid
// harmonics).  L is real-packed; returns (Re, Im) of D_x, D_y, D_z at (j, b).
template <class T>
__device__ __forceinline__ void grad_coeffs(const T *L, int j, int b, T &xr, T &xi, T &yr, T &yi, T &zr, T &zi) {
  const int n = j + 1;
  const T br = L[ridx_d(n, b, 0)], bi = b ? L[ridx_d(n, b, 1)] : T(0);
  T ar, ai;
  if (b >= 2) {
    ar = L[ridx_d(n, b - 1, 0)];
    ai = L[ridx_d(n, b - 1, 1)];
  } else if (b == 1) {
    ar = L[ridx_d(n, 0, 0)];
    ai = T(0);
  } else {  // L^{-1} = -conj(L^1)
    ar = -L[ridx_d(n, 1, 0)];
    ai = L[ridx_d(n, 1, 1)];
  }
  const T cr = L[ridx_d(n, b + 1, 0)], ci = L[ridx_d(n, b + 1, 1)];
  const T dz = (T)c_dz[j][b], r1 = (T)c_r1[j][b], r2 = (T)c_r2[j][b];
  zr = dz * br;
  zi = dz * bi;
  xr = T(0.5) * (r1 * ar - r2 * cr);
  xi = T(0.5) * (r1 * ai - r2 * ci);
  yr = T(-0.5) * (r2 * ci + r1 * ai);
  yi = T(0.5) * (r2 * cr + r1 * ar);
}

template <class T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) {
  return __builtin_amdgcn_rsqf(x);
}
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) {
  return 1.0 / sqrt(x);
}

// ---------------------------------------------------------------------------
// Bounding cube of the coordinates (open boundaries)
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_bbox_partial(const T *__restrict__ xyz, int64_t n, double *__restrict__ part) {
  __shared__ double s[6][256];
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    for (int d = 0; d < 3; ++d) {
      const double v = (double)xyz[3 * i + d];
      lo[d] = fmin(lo[d], v);
      hi[d] = fmax(hi[d], v);
    }
  for (int d = 0; d < 3; ++d) {
    s[d][threadIdx.x] = lo[d];
    s[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int d = 0; d < 3; ++d) {
        s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + w]);
        s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void k_bbox_final(const double *__restrict__ part, int nblk, Geom *g) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int b = 0; b < nblk; ++b)
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], part[b * 6 + d]);
      hi[d] = fmax(hi[d], part[b * 6 + 3 + d]);
    }
  double ext = fmax(fmax(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
  double edge = ext * (1.0 + 1e-6) + 1e-9;
  for (int d = 0; d < 3; ++d) g->origin[d] = lo[d] - 0.5 * (edge - (hi[d] - lo[d]));
  g->edge = edge;
}

// ---------------------------------------------------------------------------
// Octree build: counting sort of atoms by Morton leaf index
// ---------------------------------------------------------------------------
// Position of atom i inside the cell (w, wrapped when periodic) and its leaf
// cell c.  Divisions are replaced by products with reciprocals; an atom on a
// cell face may land in either neighbour, which the clamped leaf-local
// coordinates tolerate.
template <class T>
__device__ __forceinline__ void locate(const T *xyz, int64_t i, const Geom &g, int periodic, int n, double w[3], int c[3]) {
  const double inv_edge = 1.0 / g.edge, inv_h = n * inv_edge;
  for (int d = 0; d < 3; ++d) {
    const double x = (double)xyz[3 * i + d];
    double u;
    if (periodic) {
      u = x - g.edge * floor(x * inv_edge);
      if (u >= g.edge) u -= g.edge;
      if (u < 0.0) u = 0.0;
    } else {
      u = x - g.origin[d];
    }
    w[d] = u;
    const int ci = (int)floor(u * inv_h);
    c[d] = ci < 0 ? 0 : (ci >= n ? n - 1 : ci);
  }
}

// Leaf key of every atom, its arrival rank within the leaf (the order of
// equal keys is fixed later by k_leafsort) and its packed leaf-local
// coordinates (leaf units, centred) with the scaled charge.  Consecutive
// atoms that fall in one leaf take their ranks with a single atomic.
// Block bid of nblk (several systems of a batch each bin their own atoms;
// their keys are offset by key_off, the system's first leaf in the batch).
template <class T>
__device__ __forceinline__ void bin_body(const T *__restrict__ xyz, const T *__restrict__ qt, int64_t n_atoms,
                                         const Geom *__restrict__ gp, int d, int periodic, int *__restrict__ key,
                                         int key_off, int *__restrict__ rank, int *__restrict__ count,
                                         Atom4<T> *__restrict__ packed, Atom4<T> *__restrict__ packed_lo, int bid,
                                         int nblk) {
  const Geom g = *gp;
  const int n = 1 << d;
  const double inv_h = n / g.edge;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)nblk * blockDim.x;
  // whole waves step together (the loop bound is the same for every lane)
  for (int64_t i0 = bid * (int64_t)blockDim.x + (threadIdx.x - lane); i0 < n_atoms; i0 += stride) {
    const int64_t i = i0 + lane;
    const bool valid = i < n_atoms;
    int k = -1;
    if (valid) {
      double w[3];
      int c[3];
      locate(xyz, i, g, periodic, n, w, c);
      k = (int)morton(c[0], c[1], c[2]);
      key[i] = k + key_off;
      Atom4<T> at;
      const double lx = w[0] * inv_h - (c[0] + 0.5), ly = w[1] * inv_h - (c[1] + 0.5), lz = w[2] * inv_h - (c[2] + 0.5);
      at.x = (T)lx;
      at.y = (T)ly;
      at.z = (T)lz;
      at.q = qt[i];
      packed[i] = at;
      if (packed_lo) packed_lo[i] = Atom4<T>{(T)(lx - (double)at.x), (T)(ly - (double)at.y), (T)(lz - (double)at.z), T(0)};
    }
    // a run of equal keys on consecutive lanes (the atoms of one molecule)
    // reserves its ranks with one atomic by its first lane
    const int prev = __shfl_up(k, 1, 64);
    const bool head = lane == 0 || prev != k;
    const unsigned long long heads = __ballot(head);
    const int h = 63 - __builtin_clzll(heads & (~0ull >> (63 - lane)));
    const unsigned long long above = h == 63 ? 0ull : heads & ~(~0ull >> (63 - h));
    const int len = above ? __builtin_ctzll(above) - h : 64 - h;
    int base = 0;
    if (head && valid) base = atomicAdd(&count[k], len);
    base = __shfl(base, h, 64);
    if (valid) rank[i] = base + (lane - h);
  }
}

template <class T>
__global__ void k_bin(const T *__restrict__ xyz, const T *__restrict__ qt, int64_t n_atoms,
                      const Geom *__restrict__ gp, int d, int periodic, int *__restrict__ key, int *__restrict__ rank,
                      int *__restrict__ count, Atom4<T> *__restrict__ packed, Atom4<T> *__restrict__ packed_lo) {
  bin_body<T>(xyz, qt, n_atoms, gp, d, periodic, key, 0, rank, count, packed, packed_lo, blockIdx.x, gridDim.x);
}

// Exclusive prefix sum of the leaf counts in one block: thread t owns 32
// consecutive leaves of a round of 32,768 (eight int4 loads and stores), the
// block sums are scanned across waves.  The counts are cleared as they are
// read, ready for the binning of the next evaluation (they start cleared).
__global__ void __launch_bounds__(1024) k_scan(int *__restrict__ count, int *__restrict__ start, int nleaf) {
  constexpr int PER = 32, R = 1024 * PER;
  __shared__ int wsum[16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int carry = 0;
  for (int r0 = 0; r0 < nleaf; r0 += R) {
    const int base = r0 + t * PER;
    const bool full = base + PER <= nleaf;
    int v[PER];
    if (full) {
      int4 *c4 = reinterpret_cast<int4 *>(count + base);
#pragma unroll
      for (int i = 0; i < PER / 4; ++i) {
        const int4 x = c4[i];
        v[4 * i] = x.x;
        v[4 * i + 1] = x.y;
        v[4 * i + 2] = x.z;
        v[4 * i + 3] = x.w;
      }
#pragma unroll
      for (int i = 0; i < PER / 4; ++i) c4[i] = make_int4(0, 0, 0, 0);
    } else {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const bool in = base + k < nleaf;
        v[k] = in ? count[base + k] : 0;
        if (in) count[base + k] = 0;
      }
    }
    int loc = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) loc += v[k];
    int s = loc;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(s, o, 64);
      if (lane >= o) s += u;
    }
    if (lane == 63) wsum[wave] = s;
    __syncthreads();
    if (wave == 0) {
      int w = lane < 16 ? wsum[lane] : 0;
      for (int o = 1; o < 16; o <<= 1) {
        const int u = __shfl_up(w, o, 64);
        if (lane >= o) w += u;
      }
      if (lane < 16) wsum[lane] = w;  // inclusive prefix over waves
    }
    __syncthreads();
    int run = carry + s - loc + (wave > 0 ? wsum[wave - 1] : 0);
    if (full) {
      int4 *s4 = reinterpret_cast<int4 *>(start + base);
#pragma unroll
      for (int i = 0; i < PER / 4; ++i) {
        int4 o;
        o.x = run;
        run += v[4 * i];
        o.y = run;
        run += v[4 * i + 1];
        o.z = run;
        run += v[4 * i + 2];
        o.w = run;
        run += v[4 * i + 3];
        s4[i] = o;
      }
    } else {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        if (base + k < nleaf) start[base + k] = run;
        run += v[k];
      }
    }
    carry += wsum[15];
    __syncthreads();  // wsum is rewritten by the next round
  }
  if (t == 0) start[nleaf] = carry;
}

__global__ void k_scatter(const int *__restrict__ key, const int *__restrict__ rank, const int *__restrict__ start,
                          int *__restrict__ tmp, int64_t n_atoms) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_atoms; i += (int64_t)gridDim.x * blockDim.x)
    tmp[start[key[i]] + rank[i]] = (int)i;
}

// One wave per leaf: order the leaf's atoms by original index (deterministic
// layout), then write the permutation, its inverse and the packed atoms.
template <class T>
__global__ void __launch_bounds__(256) k_leafsort(const int *__restrict__ tmp, const int *__restrict__ start, int nleaf,
                                                  const Atom4<T> *__restrict__ packed, int *__restrict__ perm,
                                                  int *__restrict__ slot_of, Atom4<T> *__restrict__ sorted,
                                                  const Atom4<T> *__restrict__ packed_lo,
                                                  Atom4<T> *__restrict__ sorted_lo) {
  const int leaf = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (leaf >= nleaf) return;
  const int s0 = start[leaf], cnt = start[leaf + 1] - s0;
  for (int a = lane; a < cnt; a += 64) {
    const int me = tmp[s0 + a];
    int rank = 0;
    if (cnt <= 64) {
      // every atom of the leaf is held by one lane: compare through cross-lane reads
      for (int b = 0; b < cnt; ++b) rank += (__shfl(me, b, 64) < me) ? 1 : 0;
    } else {
      for (int b = 0; b < cnt; ++b) rank += (tmp[s0 + b] < me) ? 1 : 0;
    }
    const int slot = s0 + rank;
    perm[slot] = me;
    slot_of[me] = slot;
    sorted[slot] = packed[me];
    if (sorted_lo) sorted_lo[slot] = packed_lo[me];
  }
}

// ---------------------------------------------------------------------------
// P2M: leaf multipoles; also the float64 charge moments for the lattice
// ---------------------------------------------------------------------------
template <class T, int PT>
__device__ __forceinline__ void p2m_body(const Atom4<T> *__restrict__ sorted, const int *__restrict__ start, int p,
                                         int K, int KS, int chunk, T *__restrict__ Mleaf, double *__restrict__ qds,
                                         const Geom *__restrict__ gp, int d, int leaf) {
  extern __shared__ unsigned char smem_raw[];
  T *rows = reinterpret_cast<T *>(smem_raw);
  const int lane = threadIdx.x;
  const int s0 = start[leaf], cnt = start[leaf + 1] - s0;
  constexpr int kMaxPer = ((kMaxOrder + 1) * (kMaxOrder + 1) + 63) / 64;
  // float32: compensated sums (Knuth's two-sum, error terms in cmp).  A leaf's
  // monopole is a sum of ~30 charges that take a few repeated values (water
  // O and H), and plain float32 summation rounds those partial sums the same
  // way in every leaf: the bias (~1e-7 e per leaf) adds up over the tree into
  // the total charge seen by the far field and the lattice and shifts every
  // potential by a constant.  Compensated sums round each coefficient once.
  constexpr bool kComp = sizeof(T) == sizeof(float);
  T acc[kMaxPer], cmp[kMaxPer];
#pragma unroll
  for (int i = 0; i < kMaxPer; ++i) acc[i] = cmp[i] = T(0);
  for (int c0 = 0; c0 < cnt; c0 += chunk) {
    const int nch = min(chunk, cnt - c0);
    if (lane < nch) {
      const Atom4<T> a = sorted[s0 + c0 + lane];
      T *row = rows + lane * K;
      visit_regular<PT>(p, a.x, a.y, a.z, [&](int n, int m, T re, T im) {
        const int i0 = ridx_d(n, m, 0);
        row[i0] = a.q * re;
        if (m) row[i0 + 1] = -a.q * im;
      });
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
      const int k = lane + 64 * i;
      if (k < K) {
        for (int r = 0; r < nch; ++r) {
          const T v = rows[r * K + k];
          if constexpr (kComp) {
            const T t = acc[i] + v, bp = t - acc[i];
            cmp[i] += (acc[i] - (t - bp)) + (v - bp);
            acc[i] = t;
          } else {
            acc[i] += v;
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < kMaxPer; ++i) {
    const int k = lane + 64 * i;
    if (k < K) Mleaf[(int64_t)leaf * KS + k] = acc[i] + cmp[i];
  }
  if (qds) {
    const Geom g = *gp;
    const int n = 1 << d;
    const double h = g.edge / n, half = 0.5 * g.edge;
    int cx, cy, cz;
    unmorton((uint32_t)leaf, cx, cy, cz);
    double v[5] = {0, 0, 0, 0, 0};
    for (int t = lane; t < cnt; t += 64) {
      const Atom4<T> a = sorted[s0 + t];
      const double ax = (cx + 0.5 + (double)a.x) * h - half;
      const double ay = (cy + 0.5 + (double)a.y) * h - half;
      const double az = (cz + 0.5 + (double)a.z) * h - half;
      const double q = (double)a.q;
      v[0] += q;
      v[1] += q * ax;
      v[2] += q * ay;
      v[3] += q * az;
      v[4] += q * (ax * ax + ay * ay + az * az);
    }
    for (int off = 32; off > 0; off >>= 1)
      for (int k = 0; k < 5; ++k) v[k] += __shfl_xor(v[k], off);
    if (lane == 0)
      for (int k = 0; k < 5; ++k) qds[(int64_t)leaf * 5 + k] = v[k];
  }
}

template <class T, int PT>
__global__ void __launch_bounds__(64) k_p2m(const Atom4<T> *__restrict__ sorted, const int *__restrict__ start,
                                            int p, int K, int KS, int chunk, T *__restrict__ Mleaf, double *__restrict__ qds,
                                            const Geom *__restrict__ gp, int d) {
  p2m_body<T, PT>(sorted, start, p, K, KS, chunk, Mleaf, qds, gp, d, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Charge moments Q, D, S2 of the lattice remainder, first stage: block b sums
// the per-leaf moments of leaves b*256 + t, stepping over all blocks, then its
// 256 partials in a fixed tree.  Small blocks, so that the kernel runs beside
// the M2L launches instead of waiting for a free CU.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_moments(const double *__restrict__ qds, int nleaf, double *__restrict__ part) {
  __shared__ double red[5][256];
  const int t = threadIdx.x;
  double v[5] = {0, 0, 0, 0, 0};
  for (int l = blockIdx.x * 256 + t; l < nleaf; l += kMomentBlocks * 256)
    for (int k = 0; k < 5; ++k) v[k] += qds[(int64_t)l * 5 + k];
  for (int k = 0; k < 5; ++k) red[k][t] = v[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int k = 0; k < 5; ++k) red[k][t] += red[k][t + w];
    __syncthreads();
  }
  if (t < 5) part[blockIdx.x * 5 + t] = red[t][0];
}

// ---------------------------------------------------------------------------
// Periodic lattice: root local from the root multipole (float64), plus the
// float64 charge moments Q, D, S2 of the r^2 part of the lattice remainder
// (summed from nleaf rows of five moments: the block partials of k_moments).
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void lattice_body(const T *__restrict__ M, T *__restrict__ L,
                                             const double *__restrict__ LamT, int K, const double *__restrict__ qds,
                                             int nleaf, Geom *g) {
  __shared__ double red[5][1024];
  __shared__ double mroot[(kMaxOrder + 1) * (kMaxOrder + 1)];
  __shared__ double rowp[4][(kMaxOrder + 1) * (kMaxOrder + 1)];
  const int t = threadIdx.x;
  // charge moments: thread t sums leaves t, t + 1024, ... (eight in flight), then a fixed tree
  double v[5] = {0, 0, 0, 0, 0};
  int l = t;
  for (; l + 7 * 1024 < nleaf; l += 8 * 1024) {
    double r[8][5];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < 5; ++k) r[u][k] = qds[(int64_t)(l + u * 1024) * 5 + k];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < 5; ++k) v[k] += r[u][k];
  }
  for (; l < nleaf; l += 1024)
    for (int k = 0; k < 5; ++k) v[k] += qds[(int64_t)l * 5 + k];
  for (int k = 0; k < 5; ++k) red[k][t] = v[k];
  for (int c = t; c < K; c += 1024) mroot[c] = (double)M[c];
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w)
      for (int k = 0; k < 5; ++k) red[k][t] += red[k][t + w];
    __syncthreads();
  }
  if (t == 0) {
    g->Q = red[0][0];
    g->D[0] = red[1][0];
    g->D[1] = red[2][0];
    g->D[2] = red[3][0];
    g->S2 = red[4][0];
    // the root monopole is the total charge: take the float64 sum (in float32
    // the root multipole carries the rounding of every level's sums, which the
    // lattice operator would turn into a constant potential offset)
    mroot[0] = red[0][0];
  }
  __syncthreads();
  // root local = Lambda M_root: row r, column quarter q in thread (q, r); quarters summed in order
  const int q = t >> 8;
  for (int r = t & 255; r < K; r += 256) {
    const int c0 = q * K / 4, c1 = (q + 1) * K / 4;
    double acc = 0.0;
    for (int c = c0; c < c1; ++c) acc += LamT[(int64_t)c * K + r] * mroot[c];
    rowp[q][r] = acc;
  }
  __syncthreads();
  for (int rr = t; rr < K; rr += 1024) L[rr] = (T)(((rowp[0][rr] + rowp[1][rr]) + rowp[2][rr]) + rowp[3][rr]);
}

template <class T>
__global__ void __launch_bounds__(1024) k_lattice(const T *__restrict__ M, T *__restrict__ L,
                                                  const double *__restrict__ LamT, int K,
                                                  const double *__restrict__ qds, int nleaf, Geom *g) {
  lattice_body<T>(M, L, LamT, K, qds, nleaf, g);
}

// ---------------------------------------------------------------------------
// Matrix-core tile conventions (lane layouts of the A, B and D fragments) of
// the MFMA instructions used by the translation kernels.
// ---------------------------------------------------------------------------
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
template <>
struct Mfma<float> {
  static constexpr int TM = 32, TN = 32, TK = 2, NACC = 16;
  using acc_t = floatx16;
  __device__ static acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
  __device__ static int a_row(int l) { return l & 31; }
  __device__ static int a_k(int l) { return l >> 5; }
  __device__ static int b_k(int l) { return l >> 5; }
  __device__ static int b_col(int l) { return l & 31; }
  __device__ static int d_row(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
  __device__ static int d_col(int l, int) { return l & 31; }
};
template <>
struct Mfma<double> {
  static constexpr int TM = 16, TN = 16, TK = 4, NACC = 4;
  using acc_t = doublex4;
  __device__ static acc_t mma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int a_row(int l) { return l & 15; }
  __device__ static int a_k(int l) { return l >> 4; }
  __device__ static int b_k(int l) { return l >> 4; }
  __device__ static int b_col(int l) { return l & 15; }
  __device__ static int d_row(int l, int r) { return 4 * r + (l >> 4); }
  __device__ static int d_col(int l, int) { return l & 15; }
};

// float32 16x16x4 tile as used by the M2L kernel for orders up to 8: lane l
// supplies A row l % 16 and B column l % 16 of k group l / 16, and holds output
// rows 4 (l / 16) .. + 3 of column l % 16
struct Mfma16f32 {
  static constexpr int TM = 16, TN = 16, TK = 4, NACC = 4;
  typedef float acc_t __attribute__((ext_vector_type(4)));
  __device__ static acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int a_row(int l) { return l & 15; }
  __device__ static int a_k(int l) { return l >> 4; }
  __device__ static int b_k(int l) { return l >> 4; }
  __device__ static int b_col(int l) { return l & 15; }
  __device__ static int d_row(int l, int r) { return 4 * (l >> 4) + r; }
  __device__ static int d_col(int l, int) { return l & 15; }
};

constexpr int kBStride = 65;  // LDS row stride of the staged B operand (64 targets + 1 pad)

// ---------------------------------------------------------------------------
// Generic matrix-core translation: M2L, M2M and L2L as gathered GEMMs.
//   Y[target] (+)= sum_{op} T_{op} * X[source(target, op)]
// A block owns 64 targets of one parity class at one level and a group of
// output row tiles (one tile per wave, 4 waves).  For each (op, k-chunk) step
// every wave holds its operator slice in registers (prefetched one step
// ahead) and the 64 gathered source vectors sit in a double-buffered LDS
// tile, so one barrier per step suffices and global latency overlaps the
// matrix-core work of the previous step.
//   M2L: level l, 8 classes, 189 ops per class (offset lists), overwrite.
//   M2M: parent level l, 1 class, 8 ops (children), overwrite.
//   L2L: child level l, 8 classes, 1 op per class (the parent), accumulate.
// ---------------------------------------------------------------------------
enum { XL_M2L = 0, XL_M2M = 1, XL_L2L = 2 };

template <class T>
struct XChunk;
template <>
struct XChunk<float> {
  static constexpr int KC = 84;  // k values per chunk (42 MFMA steps of 2): one chunk up to order 8
};
template <>
struct XChunk<double> {
  static constexpr int KC = 44;  // 11 MFMA steps of 4
};

template <class T, int MODE, int TPT>
__global__ void __launch_bounds__(64 * TPT) k_xlate(const T *X, T *Y, const T *__restrict__ Tab,
                                               const int4 *__restrict__ ops, XArgs a) {
  using MF = Mfma<T>;
  constexpr int NCT = 64 / MF::TN;
  constexpr int KC = XChunk<T>::KC;
  constexpr int NSTEP = KC / MF::TK;
  constexpr int NB = (KC + TPT - 1) / TPT;  // staged B elements per thread and step (TPT threads per target)
  extern __shared__ unsigned char smem_raw[];
  T *Bs = reinterpret_cast<T *>(smem_raw);  // [2][KC][kBStride]

  // ---- decode the work item
  int l, li;
  if (MODE == XL_M2L) {
    l = a.lmin;
    while (l < a.d && (int)blockIdx.x >= a.level_start[l + 1]) ++l;
    li = blockIdx.x - a.level_start[l];
  } else {
    l = a.level;
    li = blockIdx.x;
  }
  const int ncls = MODE == XL_M2M ? 1 : 8;
  const int64_t ntg = MODE == XL_M2M ? (int64_t(1) << (3 * l)) : (int64_t(1) << (3 * (l - 1)));
  const int chunks = (int)((ntg + 63) / 64);
  const int g = li % a.ngroups;
  const int tq = li / a.ngroups;
  const int chunk = tq % chunks;
  const int cls = (tq / chunks) % ncls;
  const int nl = 1 << l;
  const int srclev = MODE == XL_M2L ? l : (MODE == XL_M2M ? l + 1 : l - 1);
  const int64_t xoff = level_offset(srclev), yoff = level_offset(l);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rt = g * a.nw + wave;
  const bool active = wave < a.nw && rt < a.nrt;
  const int4 *lst = ops + cls * a.nops;

  // gather mapping: thread -> (target column jt, k offset kq), TPT threads per target
  const int jt = threadIdx.x / TPT, kq = threadIdx.x - jt * TPT;
  const int64_t Pt = (int64_t)chunk * 64 + jt;
  int tx = -1, ty = -1, tz = -1;
  if (Pt < ntg) {
    if (MODE == XL_M2L) unmorton((uint32_t)(8 * Pt + cls), tx, ty, tz);
    else tx = ty = tz = 0;
  }

  const int nkc = a.KK / KC;
  const int nsteps_total = a.nops * nkc;
  T breg[NB];
  T areg[NSTEP];

  auto load_b = [&](int step) {
    const int vi = step / nkc, k0 = (step % nkc) * KC;
    const int4 v = lst[vi];
    int64_t sb = -1;
    if (tx >= 0) {
      if (MODE == XL_M2M) {
        sb = 8 * Pt + v.w;
      } else if (MODE == XL_L2L) {
        sb = Pt;
      } else {
        int sx = tx - v.x, sy = ty - v.y, sz = tz - v.z;
        bool ok = true;
        if (a.periodic) {
          sx = (sx + 4 * nl) & (nl - 1);
          sy = (sy + 4 * nl) & (nl - 1);
          sz = (sz + 4 * nl) & (nl - 1);
        } else {
          ok = (unsigned)sx < (unsigned)nl && (unsigned)sy < (unsigned)nl && (unsigned)sz < (unsigned)nl;
        }
        if (ok) sb = (int64_t)morton(sx, sy, sz);
      }
    }
    const T *src = X + (xoff + (sb < 0 ? 0 : sb)) * a.KS + k0;
    const int kmax = sb < 0 ? 0 : a.K - k0;
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int kk = kq + TPT * r;
      breg[r] = (kk < kmax && kk < KC) ? src[kk] : T(0);
    }
  };
  auto a_ptr = [&](int step) {
    const int vi = step / nkc, k0 = (step % nkc) * KC;
    const int4 v = lst[vi];
    return Tab + ((int64_t)v.w * a.KK + k0) * a.RP + rt * MF::TM + MF::a_row(lane) +
           (int64_t)MF::a_k(lane) * a.RP;
  };
  auto store_b = [&](int buf) {
    T *B = Bs + buf * KC * kBStride;
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int kk = kq + TPT * r;
      if (kk < KC) B[kk * kBStride + jt] = breg[r];
    }
  };

  typename MF::acc_t acc[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c)
#pragma unroll
    for (int r = 0; r < MF::NACC; ++r) acc[c][r] = T(0);

  load_b(0);
  if (active) {
    const T *A = a_ptr(0);
#pragma unroll
    for (int s2 = 0; s2 < NSTEP; ++s2) areg[s2] = A[(int64_t)s2 * MF::TK * a.RP];
  }
  for (int step = 0; step < nsteps_total; ++step) {
    const int buf = step & 1;
    store_b(buf);
    __syncthreads();
    const bool more = step + 1 < nsteps_total;
    if (more) load_b(step + 1);
    if (active) {
      // The chunk is full (zero-padded table rows and staged B rows), so the
      // k loop has no bounds tests and the LDS reads can run ahead of the MFMAs.
      const T *Bl = Bs + buf * KC * kBStride + MF::b_k(lane) * kBStride + MF::b_col(lane);
      const T *An = more ? a_ptr(step + 1) : a_ptr(step);
#pragma unroll
      for (int s2 = 0; s2 < NSTEP; ++s2) {
#pragma unroll
        for (int c = 0; c < NCT; ++c) acc[c] = MF::mma(areg[s2], Bl[s2 * MF::TK * kBStride + c * MF::TN], acc[c]);
        // reload this slot for the next step right after its use
        areg[s2] = An[(int64_t)s2 * MF::TK * a.RP];
      }
    }
  }
  if (active) {
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int r = 0; r < MF::NACC; ++r) {
        const int row = rt * MF::TM + MF::d_row(lane, r);
        const int col = c * MF::TN + MF::d_col(lane, r);
        const int64_t P = (int64_t)chunk * 64 + col;
        if (row < a.K && P < ntg) {
          const int64_t tb = MODE == XL_M2M ? P : 8 * P + cls;
          T *dst = Y + (yoff + tb) * a.KS + row;
          if (MODE == XL_L2L) *dst += acc[c][r];
          else *dst = acc[c][r];
        }
      }
  }
}

// ---------------------------------------------------------------------------
// M2M and L2L as stacked dense products on the vector ALU.
// The 8 children of parent P are the consecutive boxes 8P .. 8P+7 one level
// down, so for a block of NP parents:
//   M2M: M[P] = sum_c T_c M[8P + c]          (T_c: child c -> parent)
//   L2L: L[8P + c] += S_c L[P]                (S_c: parent -> child c)
// Thread (c, r) owns output row r of the child-c product for all NP parents;
// the operator element A[c][k][r] (row r fastest: coalesced) is read once and
// used for the NP parents, whose input rows sit in LDS (read as broadcasts).
// M2M sums the 8 child partials in child order through LDS; L2L adds its
// result to the child's local expansion in place (one writer per element).
// ---------------------------------------------------------------------------
template <class T, bool UP, int NP>
__device__ __forceinline__ void updown_body(T *__restrict__ X, const T *__restrict__ A, int K, int KS,
                                            int64_t off_parent, int64_t off_child, int64_t nparent, int bid) {
  extern __shared__ unsigned char smem_raw[];
  // inputs transposed so that the NP parents of one (c, k) are contiguous:
  //   UP: xs[c][k][NP] (children);  down: xs[k][NP] (parents)
  T *xs = reinterpret_cast<T *>(smem_raw);
  T *part = xs + (size_t)(UP ? 8 : 1) * KS * NP;  // UP: [NP][8][KS] child partials
  const int64_t P0 = (int64_t)bid * NP;
  const int np = (int)min((int64_t)NP, nparent - P0);
  const int in_len = UP ? 8 * KS : KS;
  {
    const T *src = UP ? X + (off_child + 8 * P0) * KS : X + (off_parent + P0) * KS;
    for (int e = threadIdx.x; e < NP * in_len; e += blockDim.x) {
      const int p = e / in_len, q = e - p * in_len;
      xs[q * NP + p] = p < np ? src[e] : T(0);
    }
  }
  __syncthreads();
  const int nrow = 8 * KS;  // (c, r) pairs
  for (int cr = threadIdx.x; cr < nrow; cr += blockDim.x) {
    const int c = cr / KS, r = cr - c * KS;
    T acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = T(0);
    const T *Ac = A + (int64_t)c * K * KS + r;
    const T *xc = xs + (UP ? c * KS * NP : 0);
    constexpr int KB = NP >= 8 ? 32 : 16;  // operator elements in flight
    for (int k0 = 0; k0 < K; k0 += KB) {
      T av[KB];
#pragma unroll
      for (int u = 0; u < KB; ++u) av[u] = k0 + u < K ? Ac[(int64_t)(k0 + u) * KS] : T(0);
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        if (k0 + u < K) {
          const T *xk = xc + (k0 + u) * NP;
#pragma unroll
          for (int p = 0; p < NP; ++p) acc[p] += av[u] * xk[p];
        }
      }
    }
    if (UP) {
#pragma unroll
      for (int p = 0; p < NP; ++p) part[(p * 8 + c) * KS + r] = acc[p];
    } else {
#pragma unroll
      for (int p = 0; p < NP; ++p)
        if (p < np && r < K) X[(off_child + 8 * (P0 + p) + c) * KS + r] += acc[p];
    }
  }
  if (UP) {
    __syncthreads();
    for (int e = threadIdx.x; e < np * KS; e += blockDim.x) {
      const int p = e / KS, r = e - p * KS;
      T s = T(0);
      for (int c = 0; c < 8; ++c) s += part[(p * 8 + c) * KS + r];
      if (r < K) X[(off_parent + P0 + p) * KS + r] = s;
    }
  }
}

template <class T, bool UP, int NP>
__global__ void __launch_bounds__(1024) k_updown(T *__restrict__ X, const T *__restrict__ A, int K, int KS,
                                                 int64_t off_parent, int64_t off_child, int64_t nparent) {
  updown_body<T, UP, NP>(X, A, K, KS, off_parent, off_child, nparent, blockIdx.x);
}

// Matrix-core tile check: C[rows x 64] = A[rows x kk] * B[kk x 64] with the same
// fragment mapping as k_xlate (A given k-major as [kk][rows]).
template <class T, class MF = Mfma<T>>
__global__ void k_mfma_probe(const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ C, int rows, int kk) {
  constexpr int NCT = 64 / MF::TN;
  const int lane = threadIdx.x & 63;
  const int rt = threadIdx.x >> 6;
  typename MF::acc_t acc[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c)
#pragma unroll
    for (int r = 0; r < MF::NACC; ++r) acc[c][r] = T(0);
  for (int kb = 0; kb < kk; kb += MF::TK) {
    const T af = A[(kb + MF::a_k(lane)) * rows + rt * MF::TM + MF::a_row(lane)];
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[c] = MF::mma(af, B[(kb + MF::b_k(lane)) * 64 + c * MF::TN + MF::b_col(lane)], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < NCT; ++c)
#pragma unroll
    for (int r = 0; r < MF::NACC; ++r)
      C[(rt * MF::TM + MF::d_row(lane, r)) * 64 + c * MF::TN + MF::d_col(lane, r)] = acc[c][r];
}

// ---------------------------------------------------------------------------
// Near field + far-field evaluation at the atoms + outputs.
// One 64-lane block per leaf (blocks of one XCD take one contiguous Morton
// range, i.e. one spatial octant, so neighbour atoms stay in that XCD's L2).
// A pass covers up to 64 targets of the leaf: each lane owns M targets (p,
// p + P, ...) and one of G source groups (every G-th source), with M chosen
// for the best lane utilisation; the G group partials are summed in group
// order with cross-lane reads.  The sources (leaf-local coordinates of their
// own leaves) are staged through LDS in the target leaf's frame as one flat
// list over the neighbourhood (p2p_wave_lds); a neighbourhood too large for
// the flat table is read straight from the sorted atoms, neighbour leaf by
// neighbour leaf, with the offset applied to the targets (p2p_wave).  Only the
// leaf itself can hold the target atom, so only its sources skip r = 0.  Then one lane per target
// evaluates the leaf's local expansion (potential and gradient; the gradient's
// coefficients are formed once per leaf), adds the r^2 part of the lattice
// remainder, and writes the potential (sorted order), the force (user order)
// and its share of the leaf's float64 energy.
// ---------------------------------------------------------------------------
struct P2PPass {
  int P, G;  // targets per group row, source groups
};

__device__ __forceinline__ P2PPass p2p_pass_shape(int nt, int mmax, int &M) {
  // lane utilisation nt * G / (64 M) for M = 1, 2, 3 (P = ceil(nt / M), G = 64 / P);
  // more targets per lane share each source load and loop step, so a larger M
  // is taken unless its utilisation is more than 0.06 below the current
  // choice's (measured on 30-atom leaves, where M = 1, 2 and 3 tie)
  int bestM = 1, bestG = 64 / max(nt, 1);
  float best = (float)nt * bestG / 64.f;
  for (int m = 2; m <= min(mmax, 3); ++m) {
    const int P = (nt + m - 1) / m;
    const int G = 64 / max(P, 1);
    const float u = (float)nt * G / (64.f * m);
    if (u >= best - 0.06f) {
      best = u;
      bestM = m;
    }
  }
  M = bestM;
  const int P = (nt + M - 1) / M;
  return {max(P, 1), 64 / max(P, 1)};
}

// FIELD = false: potential only (evaluations that return no forces).
// LO: the pair displacement from the leading parts and the rounding residuals
// of both positions, (p - o) + (p_lo - o_lo).  The leading difference of two
// nearby atoms is exact, so the displacement keeps float32 precision relative
// to its own length instead of to the leaf edge (float32 leaf-local positions
// alone carry ~2e-8 nm, which dominates the force error of close pairs once
// the expansions are accurate to order 16).
template <class T, int M, bool SELF, bool FIELD, bool LO>
__device__ __forceinline__ void p2p_pair(const Atom4<T> &o, const Atom4<T> &ol, const T (&px)[M], const T (&py)[M],
                                         const T (&pz)[M], const T (&pxl)[M], const T (&pyl)[M], const T (&pzl)[M],
                                         T (&phi)[M], T (&ex)[M], T (&ey)[M], T (&ez)[M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    T rx = px[m] - o.x, ry = py[m] - o.y, rz = pz[m] - o.z;
    if constexpr (LO) {
      rx += pxl[m] - ol.x;
      ry += pyl[m] - ol.y;
      rz += pzl[m] - ol.z;
    }
    const T r2 = rx * rx + ry * ry + rz * rz;
    T ri = rsqrt_t<T>(r2);
    if (SELF) ri = r2 > T(0) ? ri : T(0);
    const T qr = o.q * ri;
    phi[m] += qr;
    if constexpr (FIELD) {
      const T f = qr * ri * ri;
      ex[m] += f * rx;
      ey[m] += f * ry;
      ez[m] += f * rz;
    }
  }
}

// Sources s[g], s[g + G], ... of one neighbour leaf (cnt atoms), with the next
// two loaded before the current two are used (LO: with their residuals sl).
template <class T, int M, bool SELF, bool FIELD, bool LO>
__device__ __forceinline__ void p2p_run(const Atom4<T> *__restrict__ s, const Atom4<T> *__restrict__ sl, int cnt,
                                        int g, int G, const T (&px)[M], const T (&py)[M], const T (&pz)[M],
                                        const T (&pxl)[M], const T (&pyl)[M], const T (&pzl)[M], T (&phi)[M],
                                        T (&ex)[M], T (&ey)[M], T (&ez)[M]) {
  int j = g;
  if (j >= cnt) return;
  const int last = cnt - 1;
  const Atom4<T> zero{T(0), T(0), T(0), T(0)};
  Atom4<T> o0 = s[j], o1 = s[min(j + G, last)];
  Atom4<T> l0 = LO ? sl[j] : zero, l1 = LO ? sl[min(j + G, last)] : zero;
  for (; j + G < cnt; j += 2 * G) {
    const Atom4<T> n0 = s[min(j + 2 * G, last)], n1 = s[min(j + 3 * G, last)];
    Atom4<T> m0 = zero, m1 = zero;
    if constexpr (LO) {
      m0 = sl[min(j + 2 * G, last)];
      m1 = sl[min(j + 3 * G, last)];
    }
    p2p_pair<T, M, SELF, FIELD, LO>(o0, l0, px, py, pz, pxl, pyl, pzl, phi, ex, ey, ez);
    p2p_pair<T, M, SELF, FIELD, LO>(o1, l1, px, py, pz, pxl, pyl, pzl, phi, ex, ey, ez);
    o0 = n0;
    o1 = n1;
    l0 = m0;
    l1 = m1;
  }
  if (j < cnt) p2p_pair<T, M, SELF, FIELD, LO>(o0, l0, px, py, pz, pxl, pyl, pzl, phi, ex, ey, ez);
}

template <class T>
__device__ __forceinline__ T shfl_t(T v, int src) {
  return __shfl(v, src, 64);
}

// One pass: targets [tp, tp + nt) (nt <= 64) against the 27 neighbour leaves
// (start and count per neighbour in nb_st / nb_ct).  Lane u < nt receives the
// sums for target u (leaf units) in acc.
template <class T, int M, bool FIELD, bool LO>
__device__ __forceinline__ void p2p_wave(const Atom4<T> *__restrict__ sorted, const Atom4<T> *__restrict__ sorted_lo,
                                         const int *nb_st, const int *nb_ct, int tp, int nt, int lane, P2PPass ps,
                                         T (&acc)[4]) {
  const int p = lane % ps.P, g = lane / ps.P;
  T qx[M], qy[M], qz[M], qxl[M], qyl[M], qzl[M], phi[M], ex[M], ey[M], ez[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int u = p + m * ps.P;
    Atom4<T> me = {T(0), T(0), T(0), T(0)}, ml = {T(0), T(0), T(0), T(0)};
    if (u < nt) {
      me = sorted[tp + u];
      if constexpr (LO) ml = sorted_lo[tp + u];
    }
    qx[m] = me.x;
    qy[m] = me.y;
    qz[m] = me.z;
    qxl[m] = ml.x;
    qyl[m] = ml.y;
    qzl[m] = ml.z;
    phi[m] = ex[m] = ey[m] = ez[m] = T(0);
  }
  if (g < ps.G) {
    for (int r = 0; r < 27; ++r) {
      const int cnt = nb_ct[r];
      if (cnt == 0) continue;
      // target relative to the neighbour's centre: subtract the neighbour offset
      const T sx = (T)(r / 9 - 1), sy = (T)((r / 3) % 3 - 1), sz = (T)(r % 3 - 1);
      T px[M], py[M], pz[M], pxl[M], pyl[M], pzl[M];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        px[m] = qx[m] - sx;
        py[m] = qy[m] - sy;
        pz[m] = qz[m] - sz;
        if constexpr (LO) {
          // exact two-sum of the shift: p - s = px + (rounding error), plus the residual
          T bp = px[m] - qx[m];
          pxl[m] = ((qx[m] - (px[m] - bp)) + (-sx - bp)) + qxl[m];
          bp = py[m] - qy[m];
          pyl[m] = ((qy[m] - (py[m] - bp)) + (-sy - bp)) + qyl[m];
          bp = pz[m] - qz[m];
          pzl[m] = ((qz[m] - (pz[m] - bp)) + (-sz - bp)) + qzl[m];
        } else {
          pxl[m] = pyl[m] = pzl[m] = T(0);
        }
      }
      const Atom4<T> *sl = LO ? sorted_lo + nb_st[r] : nullptr;
      if (r == 13)
        p2p_run<T, M, true, FIELD, LO>(sorted + nb_st[r], sl, cnt, g, ps.G, px, py, pz, pxl, pyl, pzl, phi, ex, ey, ez);
      else
        p2p_run<T, M, false, FIELD, LO>(sorted + nb_st[r], sl, cnt, g, ps.G, px, py, pz, pxl, pyl, pzl, phi, ex, ey,
                                        ez);
    }
  }
  // lane u (target u = p' + m' P) gathers its sums from lanes g P + p' in group order
  const int pu = lane % ps.P, mu = lane / ps.P;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    for (int gg = 0; gg < ps.G; ++gg) {
      const int sl = gg * ps.P + pu;
      s0 += shfl_t(phi[m], sl);
      if constexpr (FIELD) {
        s1 += shfl_t(ex[m], sl);
        s2 += shfl_t(ey[m], sl);
        s3 += shfl_t(ez[m], sl);
      }
    }
    if (mu == m) {
      acc[0] += s0;
      acc[1] += s1;
      acc[2] += s2;
      acc[3] += s3;
    }
  }
}

// Staged near field.  The sources of a pass are the leaf itself (self pairs
// skipped) and then the other 26 neighbours as one flat list: flat source k
// belongs to neighbour slot seg[k] (a byte table built once per leaf) and sits
// at sorted index base[seg[k]] + k.  Sources are staged in LDS in the target
// leaf's frame (the neighbour offset, which also carries the periodic image
// shift, is added once per source; with residuals the shift is an exact
// two-sum), kP2PChunk at a time, with the next chunk's loads in flight while
// the current one is used.  Every lane of the wave runs the same number of
// steps, ceil(chunk / G): slots past the last source hold a zero charge far
// away.  Against one pass per neighbour this removes the per-neighbour
// rounding up of the step count (lane utilisation 0.81 -> 0.92 on ~30-atom
// leaves), the clamped global addressing of every source and the wait for
// each source's load.
constexpr int kP2PChunk = 256;
constexpr int kP2PSlots = kP2PChunk + 128;
constexpr int kP2PFlatMax = 2048;  // larger neighbourhoods take the direct path

template <class T>
struct P2PStage {
  Atom4<T> o[kP2PChunk / 64], l[kP2PChunk / 64];
  int r[kP2PChunk / 64];
};

// Loads of one chunk, branch-free (an index past the end re-reads source 0 and
// is marked empty), so that all of them are in flight together.
template <class T, bool SELF, bool LO>
__device__ __forceinline__ void p2p_stage_load(const Atom4<T> *__restrict__ sorted, const Atom4<T> *__restrict__ sorted_lo,
                                               const unsigned char *seg, const int *base, const int *rof, int total,
                                               int c, int lane, P2PStage<T> &st) {
#pragma unroll
  for (int i = 0; i < kP2PChunk / 64; ++i) {
    const int k = c * kP2PChunk + 64 * i + lane;
    const bool ok = k < total;
    const int kk = ok ? k : 0;
    const int sg = SELF ? 26 : (int)seg[kk];
    const int idx = base[sg] + kk;
    st.r[i] = ok ? rof[sg] : -1;
    st.o[i] = sorted[idx];
    if constexpr (LO) st.l[i] = sorted_lo[idx];
  }
}

template <class T, bool LO>
__device__ __forceinline__ void p2p_stage_store(const P2PStage<T> &st, int lane, Atom4<T> *buf, Atom4<T> *bufl) {
#pragma unroll
  for (int i = 0; i < kP2PChunk / 64; ++i) {
    const int r = st.r[i];
    Atom4<T> o{T(1e4), T(0), T(0), T(0)}, l{T(0), T(0), T(0), T(0)};
    if (r >= 0) {
      const T sx = (T)(r / 9 - 1), sy = (T)((r / 3) % 3 - 1), sz = (T)(r % 3 - 1);
      const Atom4<T> a = st.o[i];
      o.x = a.x + sx;
      o.y = a.y + sy;
      o.z = a.z + sz;
      o.q = a.q;
      if constexpr (LO) {
        // exact two-sum of the shift plus the stored residual
        const Atom4<T> b = st.l[i];
        T bp = o.x - a.x;
        l.x = ((a.x - (o.x - bp)) + (sx - bp)) + b.x;
        bp = o.y - a.y;
        l.y = ((a.y - (o.y - bp)) + (sy - bp)) + b.y;
        bp = o.z - a.z;
        l.z = ((a.z - (o.z - bp)) + (sz - bp)) + b.z;
      }
    }
    buf[64 * i + lane] = o;
    if constexpr (LO) bufl[64 * i + lane] = l;
  }
}

template <class T, int M, bool SELF, bool FIELD, bool LO>
__device__ __forceinline__ void p2p_segment(const Atom4<T> *__restrict__ sorted, const Atom4<T> *__restrict__ sorted_lo,
                                            const unsigned char *seg, const int *base, const int *rof, int total,
                                            int lane, int g, int G, Atom4<T> *buf, Atom4<T> *bufl, const T (&qx)[M],
                                            const T (&qy)[M], const T (&qz)[M], const T (&qxl)[M], const T (&qyl)[M],
                                            const T (&qzl)[M], T (&phi)[M], T (&ex)[M], T (&ey)[M], T (&ez)[M]) {
  const int nch = (total + kP2PChunk - 1) / kP2PChunk;
  P2PStage<T> st;
  if (nch > 0) p2p_stage_load<T, SELF, LO>(sorted, sorted_lo, seg, base, rof, total, 0, lane, st);
  for (int c = 0; c < nch; ++c) {
    __syncthreads();  // the previous chunk's reads are done
    p2p_stage_store<T, LO>(st, lane, buf, bufl);
    __syncthreads();
    if (c + 1 < nch) p2p_stage_load<T, SELF, LO>(sorted, sorted_lo, seg, base, rof, total, c + 1, lane, st);
    if (g < G) {
      const int nc = min(kP2PChunk, total - c * kP2PChunk);
      const int steps = (nc + G - 1) / G;
      const Atom4<T> zero{T(0), T(0), T(0), T(0)};
      int i = 0;
      for (; i + 1 < steps; i += 2) {
        const int j = g + i * G;
        const Atom4<T> o0 = buf[j], o1 = buf[j + G];
        const Atom4<T> l0 = LO ? bufl[j] : zero, l1 = LO ? bufl[j + G] : zero;
        p2p_pair<T, M, SELF, FIELD, LO>(o0, l0, qx, qy, qz, qxl, qyl, qzl, phi, ex, ey, ez);
        p2p_pair<T, M, SELF, FIELD, LO>(o1, l1, qx, qy, qz, qxl, qyl, qzl, phi, ex, ey, ez);
      }
      if (i < steps) {
        const int j = g + i * G;
        const Atom4<T> o0 = buf[j];
        const Atom4<T> l0 = LO ? bufl[j] : zero;
        p2p_pair<T, M, SELF, FIELD, LO>(o0, l0, qx, qy, qz, qxl, qyl, qzl, phi, ex, ey, ez);
      }
    }
  }
}

template <class T, int M, bool FIELD, bool LO>
__device__ __forceinline__ void p2p_wave_lds(const Atom4<T> *__restrict__ sorted,
                                             const Atom4<T> *__restrict__ sorted_lo, const unsigned char *seg,
                                             const int *base, const int *rof, int n_self, int n_other,
                                             Atom4<T> *buf, Atom4<T> *bufl, int tp, int nt, int lane, P2PPass ps,
                                             T (&acc)[4]) {
  const int p = lane % ps.P, g = lane / ps.P;
  T qx[M], qy[M], qz[M], qxl[M], qyl[M], qzl[M], phi[M], ex[M], ey[M], ez[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int u = p + m * ps.P;
    Atom4<T> me = {T(0), T(0), T(0), T(0)}, ml = {T(0), T(0), T(0), T(0)};
    if (u < nt) {
      me = sorted[tp + u];
      if constexpr (LO) ml = sorted_lo[tp + u];
    }
    qx[m] = me.x;
    qy[m] = me.y;
    qz[m] = me.z;
    qxl[m] = ml.x;
    qyl[m] = ml.y;
    qzl[m] = ml.z;
    phi[m] = ex[m] = ey[m] = ez[m] = T(0);
  }
  // the other 26 neighbours, then the leaf itself (table slot 26, no flat
  // table): the leaf holds most of the close pairs, whose large terms come
  // last so that the many small ones are not added to a large partial sum
  p2p_segment<T, M, false, FIELD, LO>(sorted, sorted_lo, seg, base, rof, n_other, lane, g, ps.G, buf, bufl, qx, qy,
                                      qz, qxl, qyl, qzl, phi, ex, ey, ez);
  p2p_segment<T, M, true, FIELD, LO>(sorted, sorted_lo, nullptr, base, rof, n_self, lane, g,
                                     ps.G, buf, bufl, qx, qy, qz, qxl, qyl, qzl, phi, ex, ey, ez);
  const int pu = lane % ps.P, mu = lane / ps.P;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    for (int gg = 0; gg < ps.G; ++gg) {
      const int sl = gg * ps.P + pu;
      s0 += shfl_t(phi[m], sl);
      if constexpr (FIELD) {
        s1 += shfl_t(ex[m], sl);
        s2 += shfl_t(ey[m], sl);
        s3 += shfl_t(ez[m], sl);
      }
    }
    if (mu == m) {
      acc[0] += s0;
      acc[1] += s1;
      acc[2] += s2;
      acc[3] += s3;
    }
  }
}

// Block bid handles one leaf.  perm holds atom indices of the whole batch:
// perm_off (the system's first atom) turns them into indices of F and pot_user.
template <class T, int PT, bool FIELD, bool LO>
__device__ __forceinline__ void p2p_body(const Atom4<T> *__restrict__ sorted, const Atom4<T> *__restrict__ sorted_lo,
                                         const int *__restrict__ start,
                                         const int *__restrict__ perm, int perm_off, const T *__restrict__ Lleaf,
                                         const Geom *__restrict__ gp, const P2PArgs &a, T *__restrict__ phi_sorted,
                                         T *__restrict__ F, T *__restrict__ pot_user, double *__restrict__ epart,
                                         int bid) {
  extern __shared__ unsigned char smem_raw[];
  T *loc = reinterpret_cast<T *>(smem_raw);  // [KL]: L, then (dloc) Dx, Dy, Dz
  __shared__ int nb_st[27], nb_ct[27];
  __shared__ int p2p_base[27], p2p_rof[27], p2p_tot;
  __shared__ unsigned char p2p_seg[kP2PFlatMax];
  __shared__ Atom4<T> sbuf[kP2PSlots];
  __shared__ Atom4<T> sbufl[LO ? kP2PSlots : 1];

  const int lane = threadIdx.x;
  const int n = 1 << a.d;
  const int nleaf = n * n * n;
  const int leaf = nleaf >= 8 ? (bid & 7) * (nleaf >> 3) + (bid >> 3) : bid;
  int bx = 0, by = 0, bz = 0;
  unmorton((uint32_t)leaf, bx, by, bz);

  if (lane < 27) {
    int cx = bx - 1 + lane / 9, cy = by - 1 + (lane / 3) % 3, cz = bz - 1 + lane % 3;
    bool ok = true;
    if (a.periodic) {
      cx = (cx + n) % n;
      cy = (cy + n) % n;
      cz = (cz + n) % n;
    } else {
      ok = (unsigned)cx < (unsigned)n && (unsigned)cy < (unsigned)n && (unsigned)cz < (unsigned)n;
    }
    int st = 0, cnt = 0;
    if (ok) {
      const int nb = (int)morton(cx, cy, cz);
      st = start[nb];
      cnt = start[nb + 1] - st;
    }
    nb_st[lane] = st;
    nb_ct[lane] = cnt;
  }
  for (int e = lane; e < a.K; e += 64) loc[e] = Lleaf[(int64_t)leaf * a.KS + e];
  // permanent far-away zero-charge slots past the chunk (steps run past the last source)
  for (int e = kP2PChunk + lane; e < kP2PSlots; e += 64) {
    sbuf[e] = Atom4<T>{T(1e4), T(0), T(0), T(0)};
    if constexpr (LO) sbufl[e] = Atom4<T>{T(0), T(0), T(0), T(0)};
  }
  __syncthreads();
  // flat source tables: slots 0..25 the other neighbours in order, slot 26 the leaf itself
  {
    int acc = 0;
    for (int sg = 0; sg < 26; ++sg) {
      const int r = sg < 13 ? sg : sg + 1;
      const int cnt = nb_ct[r];
      if (lane == 0) {
        p2p_base[sg] = nb_st[r] - acc;
        p2p_rof[sg] = r;
      }
      for (int k = acc + lane; k < acc + cnt && k < kP2PFlatMax; k += 64) p2p_seg[k] = (unsigned char)sg;
      acc += cnt;
    }
    if (lane == 0) {
      p2p_base[26] = nb_st[13];
      p2p_rof[26] = 13;
      p2p_tot = acc;
    }
  }
  if (FIELD && a.dloc) {
    // gradient coefficients Dx, Dy, Dz in the real packing of L (degrees < p)
    const int nd = a.p * a.p;
    for (int k = lane; k < nd; k += 64) {
      int j = 0;
      while ((j + 1) * (j + 1) <= k) ++j;
      const int r = k - j * j;  // 0 -> m = 0; then (m, re), (m, im) pairs
      const int b = (r + 1) >> 1;
      const bool imag = r > 0 && (r & 1) == 0;
      T xr, xi, yr, yi, zr, zi;
      grad_coeffs(loc, j, b, xr, xi, yr, yi, zr, zi);
      loc[a.K + k] = imag ? xi : xr;
      loc[2 * a.K + k] = imag ? yi : yr;
      loc[3 * a.K + k] = imag ? zi : zr;
    }
  }
  __syncthreads();

  const Geom g = *gp;
  const double h = g.edge / n, inv_h = 1.0 / h, half = 0.5 * g.edge;
  const double c_r2 = a.periodic ? 2.0 * 3.14159265358979323846 / (3.0 * g.edge * g.edge * g.edge) : 0.0;
  const int tb = nb_st[13], nt_leaf = nb_ct[13];
  const T *Dx = loc + a.K, *Dy = Dx + a.K, *Dz = Dy + a.K;
  double esum = 0.0;
  for (int tp = tb; tp < tb + nt_leaf; tp += 64) {
    const int nt = min(64, tb + nt_leaf - tp);
    int M;
    const P2PPass ps = p2p_pass_shape(nt, a.mmax, M);
    T acc[4] = {T(0), T(0), T(0), T(0)};
    if (p2p_tot <= kP2PFlatMax) {
      if (M == 1)
        p2p_wave_lds<T, 1, FIELD, LO>(sorted, sorted_lo, p2p_seg, p2p_base, p2p_rof, nt_leaf, p2p_tot, sbuf, sbufl,
                                      tp, nt, lane, ps, acc);
      else if (M == 2)
        p2p_wave_lds<T, 2, FIELD, LO>(sorted, sorted_lo, p2p_seg, p2p_base, p2p_rof, nt_leaf, p2p_tot, sbuf, sbufl,
                                      tp, nt, lane, ps, acc);
      else
        p2p_wave_lds<T, 3, FIELD, LO>(sorted, sorted_lo, p2p_seg, p2p_base, p2p_rof, nt_leaf, p2p_tot, sbuf, sbufl,
                                      tp, nt, lane, ps, acc);
    } else {
      // neighbourhoods beyond the flat table: one pass per neighbour from global memory
      if (M == 1) p2p_wave<T, 1, FIELD, LO>(sorted, sorted_lo, nb_st, nb_ct, tp, nt, lane, ps, acc);
      else if (M == 2) p2p_wave<T, 2, FIELD, LO>(sorted, sorted_lo, nb_st, nb_ct, tp, nt, lane, ps, acc);
      else p2p_wave<T, 3, FIELD, LO>(sorted, sorted_lo, nb_st, nb_ct, tp, nt, lane, ps, acc);
    }
    if (lane < nt) {
      const int ti = tp + lane;
      const Atom4<T> me = sorted[ti];
      T pf = T(0), gx = T(0), gy = T(0), gz = T(0);
      const int p = PT > 0 ? PT : a.p;
      if constexpr (!FIELD) {
        visit_regular<PT>(p, me.x, me.y, me.z, [&](int nn, int m, T re, T im) {
          const int i0 = ridx_d(nn, m, 0);
          if (m) pf += T(2) * (loc[i0] * re + loc[i0 + 1] * im);
          else pf += loc[i0] * re;
        });
      } else if (a.dloc) {
        visit_regular<PT>(p, me.x, me.y, me.z, [&](int nn, int m, T re, T im) {
          const int i0 = ridx_d(nn, m, 0);
          if (m) {
            pf += T(2) * (loc[i0] * re + loc[i0 + 1] * im);
            if (nn < p) {
              gx += T(2) * (Dx[i0] * re + Dx[i0 + 1] * im);
              gy += T(2) * (Dy[i0] * re + Dy[i0 + 1] * im);
              gz += T(2) * (Dz[i0] * re + Dz[i0 + 1] * im);
            }
          } else {
            pf += loc[i0] * re;
            if (nn < p) {
              gx += Dx[i0] * re;
              gy += Dy[i0] * re;
              gz += Dz[i0] * re;
            }
          }
        });
      } else {
        for_regular(p, me.x, me.y, me.z, [&](int nn, int m, T re, T im) {
          const int i0 = ridx_d(nn, m, 0);
          const T w = m ? T(2) : T(1);
          pf += w * (loc[i0] * re + (m ? loc[i0 + 1] * im : T(0)));
          if (nn < p) {
            T xr, xi, yr, yi, zr, zi;
            grad_coeffs(loc, nn, m, xr, xi, yr, yi, zr, zi);
            gx += w * (xr * re + xi * im);
            gy += w * (yr * re + yi * im);
            gz += w * (zr * re + zi * im);
          }
        });
      }
      double ph = ((double)acc[0] + (double)pf) * inv_h;
      double E[3] = {((double)acc[1] - (double)gx) * inv_h * inv_h, ((double)acc[2] - (double)gy) * inv_h * inv_h,
                     ((double)acc[3] - (double)gz) * inv_h * inv_h};
      if (a.periodic) {
        const double ax = (bx + 0.5 + (double)me.x) * h - half;
        const double ay = (by + 0.5 + (double)me.y) * h - half;
        const double az = (bz + 0.5 + (double)me.z) * h - half;
        ph += c_r2 * (g.Q * (ax * ax + ay * ay + az * az) - 2.0 * (g.D[0] * ax + g.D[1] * ay + g.D[2] * az) + g.S2);
        E[0] += 2.0 * c_r2 * (g.D[0] - g.Q * ax);
        E[1] += 2.0 * c_r2 * (g.D[1] - g.Q * ay);
        E[2] += 2.0 * c_r2 * (g.D[2] - g.Q * az);
      }
      const double q = (double)me.q;
      phi_sorted[ti] = (T)ph;
      const int64_t u = perm[ti] - perm_off;
      if (FIELD && F) {
        F[3 * u + 0] = (T)(a.ke * q * E[0]);
        F[3 * u + 1] = (T)(a.ke * q * E[1]);
        F[3 * u + 2] = (T)(a.ke * q * E[2]);
      }
      if (pot_user) pot_user[u] = (T)(a.ke * ph);
      esum += q * ph;
    }
  }
  for (int off = 32; off > 0; off >>= 1) esum += __shfl_xor(esum, off);
  if (lane == 0) epart[leaf] = esum;
}

template <class T, int PT, bool FIELD, bool LO>
__global__ void __launch_bounds__(64) k_p2p_l2p(const Atom4<T> *__restrict__ sorted,
                                                const Atom4<T> *__restrict__ sorted_lo, const int *__restrict__ start,
                                                const int *__restrict__ perm, const T *__restrict__ Lleaf,
                                                const Geom *__restrict__ gp, P2PArgs a, T *__restrict__ phi_sorted,
                                                T *__restrict__ F, T *__restrict__ pot_user,
                                                double *__restrict__ epart) {
  p2p_body<T, PT, FIELD, LO>(sorted, sorted_lo, start, perm, 0, Lleaf, gp, a, phi_sorted, F, pot_user, epart,
                             blockIdx.x);
}

// ---------------------------------------------------------------------------
// Charge scaling (paper, eq after eq constraint): qt = sum_r lt_r q^(s,r) at site atoms.
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_charge_scale(const int *__restrict__ atom_off, const int *__restrict__ form_off,
                               const int *__restrict__ site_atoms, const double *__restrict__ fq,
                               const int *__restrict__ fq_off, const double *__restrict__ lam, int n_sites,
                               T *__restrict__ qt) {
  const int s = blockIdx.x;
  if (s >= n_sites) return;
  const int na = atom_off[s + 1] - atom_off[s], nf = form_off[s + 1] - form_off[s];
  for (int i = threadIdx.x; i < na; i += blockDim.x) {
    double v = 0.0;
    for (int r = 0; r < nf; ++r) v += lam[form_off[s] + r] * fq[fq_off[s] + r * na + i];
    qt[site_atoms[atom_off[s] + i]] = (T)v;
  }
}

// ---------------------------------------------------------------------------
// MAHI site correction, float64, one block of 64 threads per site.
// Site kernel Phi_ij = sum over the 27 nearest images of 1/|r_ij + nL| (the
// "box-box" part, computed directly as in an FMM of depth 0) + the truncated
// lattice bilinear form that the tree applied to the pair + the r^2 part; the
// same wrapped coordinates as the tree are used so that the correction
// removes the tree's intra-site terms.  With U^r_i = sum_j Phi_ij q^r_j and
// Ut = sum_r lt_r U^r (the site's own share of the scaled potential):
//   C^r   = sum_i q^r_i (Ut_i - U^r_i / 2)                (correction, eq correction_scheme)
//   dV/dlt_r = ke (sum_i q^r_i V_i - C^r)                  (per-form part of the mapping K)
//   dE_s  = 1/2 (sum_r lt_r q^r.U^r - qt.Ut)               (HI minus charge-scaled intra-site energy)
//   dF_i  = sum_r lt_r q^r_i W^r_i - qt_i Wt_i,  W = sum_j G_ij q_j, G = -grad_i Phi
// and, with every weight and form charge an independent variable (general
// formulation, eq iter_ham_lambda),
//   dE/dq^r_i = ke lt_r (V_i + U^r_i - Ut_i)
//   dE_QI/dlt_r = ke sum_i q^r_i V_i     (charge interpolation: E_QI = ke/2 qt.Phi.qt)
// ---------------------------------------------------------------------------
template <class T, int PT, bool WS>
__device__ __forceinline__ void site_body(const SiteArgs &a, const T *__restrict__ xyz, const int *__restrict__ slot_of,
                                          const Geom *__restrict__ gp, const double *__restrict__ LamT,
                                          const SiteIO<T> &io, int s) {
  T *__restrict__ F = io.F;
  constexpr int NT = 256;
  extern __shared__ double sm_lds[];
  const int tid = threadIdx.x;
  // work arrays in local memory, or (WS) this site's region of the global workspace;
  // a compile-time choice, so that the local-memory case keeps LDS instructions
  double *sm = WS ? io.ws + (size_t)s * io.ws_stride : sm_lds;
  const int na = a.atom_off[s + 1] - a.atom_off[s], nf = a.form_off[s + 1] - a.form_off[s];
  const int K = a.K, p = PT > 0 ? PT : a.p;
  __shared__ double x[kMaxSiteAtoms][3], V[kMaxSiteAtoms], qt[kMaxSiteAtoms], ut[kMaxSiteAtoms], lam[kMaxSiteForms];
  __shared__ double qf[kMaxSiteForms][kMaxSiteAtoms];
  __shared__ double U[kMaxSiteForms][kMaxSiteAtoms], W[kMaxSiteForms][kMaxSiteAtoms][3];
  // dynamic: PG[maxa][maxa][4] (pair kernel Phi and G), Rt[maxa][K] (unconjugated Rt at
  // (x - c)/L), om[maxf][K] (site multipoles), Lat[maxf][LS] (lattice locals, followed by their
  // gradient coefficients Dx, Dy, Dz when a.dloc: LS = 4K, else LS = K)
  const int LS = a.dloc ? 4 * K : K;
  double *PG = sm;
  double *Rt = PG + (size_t)4 * a.maxa * a.maxa;
  double *om = Rt + (size_t)a.maxa * K;
  double *Lat = om + (size_t)a.maxf * K;

  const Geom g = *gp;
  const double L = g.edge;
  if (tid < na) {
    const int atom = a.site_atoms[a.atom_off[s] + tid];
    for (int d = 0; d < 3; ++d) {
      const double xv = (double)xyz[3 * (int64_t)atom + d];
      x[tid][d] = a.periodic ? wrap_coord(xv, L) : xv;
    }
    V[tid] = io.pot_ext ? (double)io.pot_ext[atom] / a.ke : (double)io.phi_sorted[slot_of[atom]];
  }
  if (tid < nf) lam[tid] = a.lam[a.form_off[s] + tid];
  for (int e = tid; e < nf * na; e += NT) {
    const int r = e / na, i = e % na;
    qf[r][i] = a.fq[a.fq_off[s] + r * na + i];
  }
  __syncthreads();
  if (tid < na) {
    double v = 0.0;
    for (int r = 0; r < nf; ++r) v += lam[r] * qf[r][tid];
    qt[tid] = v;
  }
  // pair kernel over the 27 nearest images (+ r^2 part when periodic), once per atom pair:
  // PG[i][j] = (Phi_ij, G_ij) with G = -grad_i Phi
  const double c_r2 = a.periodic ? 2.0 * 3.14159265358979323846 / (3.0 * L * L * L) : 0.0;
  const int R = a.periodic ? 1 : 0;
  for (int e = tid; e < na * na; e += NT) {
    const int i = e / na, j = e % na;
    const double rx = x[i][0] - x[j][0], ry = x[i][1] - x[j][1], rz = x[i][2] - x[j][2];
    double ph = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int ia = -R; ia <= R; ++ia)
      for (int ib = -R; ib <= R; ++ib)
        for (int ic = -R; ic <= R; ++ic) {
          if (i == j && ia == 0 && ib == 0 && ic == 0) continue;
          const double dx = rx + ia * L, dy = ry + ib * L, dz = rz + ic * L;
          const double ri = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
          ph += ri;
          const double f = ri * ri * ri;
          gx += f * dx;
          gy += f * dy;
          gz += f * dz;
        }
    if (a.periodic) {
      ph += c_r2 * (rx * rx + ry * ry + rz * rz);
      gx -= 2.0 * c_r2 * rx;
      gy -= 2.0 * c_r2 * ry;
      gz -= 2.0 * c_r2 * rz;
    }
    double *pg = PG + (size_t)e * 4;
    pg[0] = ph;
    pg[1] = gx;
    pg[2] = gy;
    pg[3] = gz;
  }
  __syncthreads();
  for (int e = tid; e < nf * na; e += NT) {
    const int r = e / na, i = e % na;
    double u = 0.0, w0 = 0.0, w1 = 0.0, w2 = 0.0;
    for (int j = 0; j < na; ++j) {
      const double *pg = PG + (size_t)(i * na + j) * 4;
      const double qj = qf[r][j];
      u += pg[0] * qj;
      w0 += pg[1] * qj;
      w1 += pg[2] * qj;
      w2 += pg[3] * qj;
    }
    U[r][i] = u;
    W[r][i][0] = w0;
    W[r][i][1] = w1;
    W[r][i][2] = w2;
  }
  if (a.periodic) {
    // lattice part: the tree's truncated lattice operator applied to the site's own charges
    const double half = 0.5 * L, invL = 1.0 / L;
    if (tid < na) {
      double *row = Rt + tid * K;
      visit_regular<PT>(p, (x[tid][0] - half) * invL, (x[tid][1] - half) * invL, (x[tid][2] - half) * invL,
                        [&](int n, int m, double re, double im) {
                          const int i0 = ridx_d(n, m, 0);
                          row[i0] = re;
                          if (m) row[i0 + 1] = im;
                        });
    }
    __syncthreads();
    for (int e = tid; e < nf * K; e += NT) {
      const int r = e / K, k = e % K;
      // multipole = sum q conj(Rt): the imaginary slots (even, nonzero offset within a degree) flip sign
      int nd = 0;
      while ((nd + 1) * (nd + 1) <= k) ++nd;
      const int o = k - nd * nd;
      const double sgn = (o > 0 && (o & 1) == 0) ? -1.0 : 1.0;
      double v = 0.0;
      for (int i = 0; i < na; ++i) v += qf[r][i] * Rt[i * K + k];
      om[r * K + k] = sgn * v;
    }
    __syncthreads();
    for (int e = tid; e < nf * K; e += NT) {
      const int r = e / K, k = e % K;
      const double *orr = om + r * K;
      double v = 0.0;
      int c = 0;
      for (; c + 8 <= K; c += 8) {
        double l8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) l8[u] = LamT[(int64_t)(c + u) * K + k];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += l8[u] * orr[c + u];
      }
      for (; c < K; ++c) v += LamT[(int64_t)c * K + k] * orr[c];
      Lat[(size_t)r * LS + k] = v;
    }
    __syncthreads();
    // gradient coefficients of each form's lattice local (degrees < p)
    const int nd = a.dloc ? p * p : 0;
    for (int e = tid; e < nf * nd; e += NT) {
      const int r = e / nd, k = e % nd;
      int j = 0;
      while ((j + 1) * (j + 1) <= k) ++j;
      const int o = k - j * j;
      const int b = (o + 1) >> 1;
      const bool imag = o > 0 && (o & 1) == 0;
      double xr, xi, yr, yi, zr, zi;
      double *Lr = Lat + (size_t)r * LS;
      grad_coeffs(Lr, j, b, xr, xi, yr, yi, zr, zi);
      Lr[K + k] = imag ? xi : xr;
      Lr[2 * K + k] = imag ? yi : yr;
      Lr[3 * K + k] = imag ? zi : zr;
    }
    __syncthreads();
    for (int e = tid; e < nf * na; e += NT) {
      const int r = e / na, i = e % na;
      const double *Rr = Rt + i * K;
      const double *Lr = Lat + (size_t)r * LS;
      const double *Dx = Lr + K, *Dy = Dx + K, *Dz = Dy + K;
      double pot = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
      for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
          const int i0 = ridx_d(n, m, 0);
          const double w = m ? 2.0 : 1.0;
          const double rre = Rr[i0], rim = m ? Rr[i0 + 1] : 0.0;
          pot += w * (Lr[i0] * rre + (m ? Lr[i0 + 1] * rim : 0.0));
          if (n < p) {
            double xr, xi, yr, yi, zr, zi;
            if (a.dloc) {
              xr = Dx[i0], yr = Dy[i0], zr = Dz[i0];
              xi = m ? Dx[i0 + 1] : 0.0, yi = m ? Dy[i0 + 1] : 0.0, zi = m ? Dz[i0 + 1] : 0.0;
            } else {
              grad_coeffs(Lr, n, m, xr, xi, yr, yi, zr, zi);
            }
            gx += w * (xr * rre + xi * rim);
            gy += w * (yr * rre + yi * rim);
            gz += w * (zr * rre + zi * rim);
          }
        }
      U[r][i] += pot * invL;
      W[r][i][0] -= gx * invL * invL;
      W[r][i][1] -= gy * invL * invL;
      W[r][i][2] -= gz * invL * invL;
    }
  }
  __syncthreads();
  // per-atom combination and force correction
  if (tid < na) {
    double u = 0.0, wt0 = 0.0, wt1 = 0.0, wt2 = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int r = 0; r < nf; ++r) {
      u += lam[r] * U[r][tid];
      wt0 += lam[r] * W[r][tid][0];
      wt1 += lam[r] * W[r][tid][1];
      wt2 += lam[r] * W[r][tid][2];
      d0 += lam[r] * qf[r][tid] * W[r][tid][0];
      d1 += lam[r] * qf[r][tid] * W[r][tid][1];
      d2 += lam[r] * qf[r][tid] * W[r][tid][2];
    }
    d0 -= qt[tid] * wt0;
    d1 -= qt[tid] * wt1;
    d2 -= qt[tid] * wt2;
    const int64_t atom = a.site_atoms[a.atom_off[s] + tid];
    if (F) {
      F[3 * atom + 0] = (T)((double)F[3 * atom + 0] + a.ke * d0);
      F[3 * atom + 1] = (T)((double)F[3 * atom + 1] + a.ke * d1);
      F[3 * atom + 2] = (T)((double)F[3 * atom + 2] + a.ke * d2);
    }
    ut[tid] = u;
  }
  __syncthreads();
  if (tid < nf) {
    const int r = tid;
    double c = 0.0, vq = 0.0;
    for (int i = 0; i < na; ++i) {
      c += qf[r][i] * (ut[i] - 0.5 * U[r][i]);
      vq += qf[r][i] * V[i];
    }
    if (io.dvdl) io.dvdl[a.form_off[s] + r] = a.ke * (vq - c);
    if (io.dvdl_qi) io.dvdl_qi[a.form_off[s] + r] = a.ke * vq;
  }
  if (io.dedq)
    for (int e = tid; e < nf * na; e += NT) {
      const int r = e / na, i = e % na;
      io.dedq[a.fq_off[s] + e] = a.ke * lam[r] * (V[i] + U[r][i] - ut[i]);
    }
  if (tid == 0) {
    double e = 0.0;
    for (int r = 0; r < nf; ++r) {
      double t = 0.0;
      for (int i = 0; i < na; ++i) t += qf[r][i] * U[r][i];
      e += lam[r] * t;
    }
    for (int i = 0; i < na; ++i) e -= qt[i] * ut[i];
    io.dE_site[s] = 0.5 * e;
  }
}

template <class T, int PT, bool WS>
__global__ void __launch_bounds__(256) k_site(SiteArgs a, const T *__restrict__ xyz, const int *__restrict__ slot_of,
                                              const Geom *__restrict__ gp, const double *__restrict__ LamT,
                                              SiteIO<T> io) {
  site_body<T, PT, WS>(a, xyz, slot_of, gp, LamT, io, blockIdx.x);
}

// E = ke (1/2 sum_blocks epart + sum_sites dE) and, when E_qi is set, the
// charge-interpolated energy ke/2 sum_blocks epart; fixed order.
__device__ __forceinline__ void finalize_body(const double *__restrict__ epart, int nb,
                                              const double *__restrict__ dE_site, int ns, double ke,
                                              double *__restrict__ E, double *__restrict__ E_qi) {
  __shared__ double s[1024], sq[1024];
  const int t = threadIdx.x;
  // fixed-order partial sums: thread t adds entries t, t + 1024, ... (loads unrolled 8-fold)
  double v = 0.0, w = 0.0;
  int i = t;
  for (; i + 7 * 1024 < nb; i += 8 * 1024) {
    double r[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = epart[i + k * 1024];
#pragma unroll
    for (int k = 0; k < 8; ++k) v += r[k];
  }
  for (; i < nb; i += 1024) v += epart[i];
  for (int k = t; k < ns; k += 1024) w += dE_site[k];
  s[t] = 0.5 * v + w;
  sq[t] = 0.5 * v;
  __syncthreads();
  for (int k = 512; k > 0; k >>= 1) {
    if (t < k) {
      s[t] += s[t + k];
      sq[t] += sq[t + k];
    }
    __syncthreads();
  }
  if (t == 0) {
    *E = ke * s[0];
    if (E_qi) *E_qi = ke * sq[0];
  }
}

__global__ void __launch_bounds__(1024) k_finalize(const double *__restrict__ epart, int nb,
                                                   const double *__restrict__ dE_site, int ns, double ke,
                                                   double *__restrict__ E, double *__restrict__ E_qi) {
  finalize_body(epart, nb, dE_site, ns, ke, E, E_qi);
}

// ---------------------------------------------------------------------------
// Packed batch kernels: the single-system stages above, one launch over all
// systems of a batch.  Each block finds its system by a binary search of the
// stage's block ranges and runs the same body with that system's offsets.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int packed_system(const int *__restrict__ first, int nsys, int b) {
  int lo = 0, hi = nsys;  // largest s with first[s] <= b (a system with blocks)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void kp_bin(const PackedSys *__restrict__ sys, const int *__restrict__ first, int nsys,
                       int *__restrict__ key, int *__restrict__ rank, int *__restrict__ count,
                       Atom4<float> *__restrict__ packed) {
  const int s = packed_system(first, nsys, blockIdx.x);
  const PackedSys &S = sys[s];
  bin_body<float>(S.xyz, S.qt, S.n_atoms, S.geom, S.d, 1, key + S.atom_off, S.leaf_off, rank + S.atom_off,
                  count + S.leaf_off, packed + S.atom_off, nullptr, blockIdx.x - first[s], first[s + 1] - first[s]);
}

template <int PT>
__global__ void __launch_bounds__(64) kp_p2m(const PackedSys *__restrict__ sys, const int *__restrict__ first,
                                             int nsys, const Atom4<float> *__restrict__ sorted,
                                             const int *__restrict__ start, int p, int K, int KS, int chunk,
                                             float *__restrict__ Mc, double *__restrict__ qds) {
  const int s = packed_system(first, nsys, blockIdx.x);
  const PackedSys &S = sys[s];
  p2m_body<float, PT>(sorted, start + S.leaf_off, p, K, KS, chunk, Mc + (S.box_off + level_offset(S.d)) * KS,
                      qds + (int64_t)S.leaf_off * 5, S.geom, S.d, blockIdx.x - first[s]);
}

// M2M (UP, parent level d - step) or L2L (parent level step - 1) of every system
template <bool UP, int NP>
__global__ void __launch_bounds__(1024) kp_updown(const PackedSys *__restrict__ sys, const int *__restrict__ first,
                                                  int nsys, float *__restrict__ X, const float *__restrict__ A, int K,
                                                  int KS, int step) {
  const int s = packed_system(first, nsys, blockIdx.x);
  const PackedSys &S = sys[s];
  const int pl = UP ? S.d - step : step - 1;
  updown_body<float, UP, NP>(X + S.box_off * KS, A, K, KS, level_offset(pl), level_offset(pl + 1),
                             int64_t(1) << (3 * pl), blockIdx.x - first[s]);
}

__global__ void __launch_bounds__(1024) kp_lattice(const PackedSys *__restrict__ sys, const float *__restrict__ Mc,
                                                   float *__restrict__ Lc, const double *__restrict__ LamT, int K,
                                                   int KS, const double *__restrict__ qds) {
  const PackedSys &S = sys[blockIdx.x];
  lattice_body<float>(Mc + S.box_off * KS, Lc + S.box_off * KS, LamT, K, qds + (int64_t)S.leaf_off * 5, S.nleaf,
                      S.geom);
}

template <int PT>
__global__ void __launch_bounds__(64) kp_p2p(const PackedSys *__restrict__ sys, const int *__restrict__ first,
                                             int nsys, const Atom4<float> *__restrict__ sorted,
                                             const int *__restrict__ start, const int *__restrict__ perm,
                                             const float *__restrict__ Lc, int KS, float *__restrict__ phi_sorted,
                                             double *__restrict__ epart) {
  const int s = packed_system(first, nsys, blockIdx.x);
  const PackedSys &S = sys[s];
  p2p_body<float, PT, true, false>(sorted, nullptr, start + S.leaf_off, perm, (int)S.atom_off,
                                   Lc + (S.box_off + level_offset(S.d)) * KS, S.geom, S.p2p, phi_sorted, S.F,
                                   S.pot, epart + S.leaf_off, blockIdx.x - first[s]);
}

template <int PT>
__global__ void __launch_bounds__(256) kp_site(const PackedSys *__restrict__ sys, const int *__restrict__ first,
                                               int nsys, const int *__restrict__ slot_of,
                                               const double *__restrict__ LamT) {
  const int s = packed_system(first, nsys, blockIdx.x);
  const PackedSys &S = sys[s];
  site_body<float, PT, false>(S.site, S.xyz, slot_of + S.atom_off, S.geom, LamT, S.io, blockIdx.x - first[s]);
}

__global__ void __launch_bounds__(1024) kp_finalize(const PackedSys *__restrict__ sys,
                                                    const double *__restrict__ epart) {
  const PackedSys &S = sys[blockIdx.x];
  finalize_body(epart + S.leaf_off, S.nleaf, S.io.dE_site, S.n_sites, S.ke, S.E, S.E_qi);
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free correction: per-site energies and the
// site pass's work arrays of one call.  Every device the library runs on holds
// its own copy for the life of the process.  In host code `scratch` is only a
// stand-in for the symbol: its device address comes from hipGetSymbolAddress
// and is kept per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(int device, void **ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static inline int grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  if (g > 65535 * 8) g = 65535 * 8;
  if (g < 1) g = 1;
  return (int)g;
}

template <class T>
void launch_bbox(const T *xyz, int64_t n, double *part, int nblk, Geom *g, hipStream_t st) {
  hipLaunchKernelGGL(k_bbox_partial<T>, dim3(nblk), dim3(256), 0, st, xyz, n, part);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, part, nblk, g);
}

template <class T>
void launch_tree(const T *xyz, const T *qt, int64_t n, const Geom *g, int d, int periodic, TreeBufs<T> b,
                 hipStream_t st) {
  const int nleaf = 1 << (3 * d);
  // slot_of holds the in-leaf arrival ranks until k_leafsort writes the slots;
  // count is zero on entry (cleared at creation and by every k_scan)
  hipLaunchKernelGGL(k_bin<T>, dim3(grid_for(n, 256)), dim3(256), 0, st, xyz, qt, n, g, d, periodic, b.key, b.slot_of,
                     b.count, b.packed, b.packed_lo);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, b.count, b.start, nleaf);
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, 256)), dim3(256), 0, st, b.key, b.slot_of, b.start, b.tmp, n);
  hipLaunchKernelGGL(k_leafsort<T>, dim3((nleaf + 3) / 4), dim3(256), 0, st, b.tmp, b.start, nleaf, b.packed, b.perm,
                     b.slot_of, b.sorted, b.packed_lo, b.sorted_lo);
}

template <class T>
void launch_p2m(const Atom4<T> *sorted, const int *start, int nleaf, int p, int KS, T *Mleaf, double *qds, const Geom *g,
                int d, hipStream_t st) {
  const int K = (p + 1) * (p + 1);
  // atoms per LDS pass: at most 32 (a typical leaf in one pass, small enough
  // LDS for many one-wave blocks per CU)
  int chunk = (int)(16384 / (K * sizeof(T)));
  if (chunk > 32) chunk = 32;
  if (chunk < 1) chunk = 1;
  if (p == 8)
    hipLaunchKernelGGL((k_p2m<T, 8>), dim3(nleaf), dim3(64), chunk * K * sizeof(T), st, sorted, start, p, K, KS, chunk,
                       Mleaf, qds, g, d);
  else
    hipLaunchKernelGGL((k_p2m<T, 0>), dim3(nleaf), dim3(64), chunk * K * sizeof(T), st, sorted, start, p, K, KS, chunk,
                       Mleaf, qds, g, d);
}

void launch_moments(const double *qds, int nleaf, double *part, hipStream_t st) {
  hipLaunchKernelGGL(k_moments, dim3(kMomentBlocks), dim3(256), 0, st, qds, nleaf, part);
}

template <class T>
void launch_lattice(const T *M, T *L, const double *LamT, int K, const double *part, Geom *g, hipStream_t st) {
  hipLaunchKernelGGL(k_lattice<T>, dim3(1), dim3(1024), 0, st, M, L, LamT, K, part, kMomentBlocks, g);
}

// Operator tables: [slot][KK][RP], k padded with zero rows to whole chunks of
// XChunk<T>::KC and rows padded to whole MFMA row tiles.
template <class T>
void m2l_table_layout(int p, int &KK, int &RP) {
  using MF = Mfma<T>;
  constexpr int KC = XChunk<T>::KC;
  const int K = (p + 1) * (p + 1);
  KK = (K + KC - 1) / KC * KC;
  RP = (K + MF::TM - 1) / MF::TM * MF::TM;
}

template <class T>
void xlate_geometry(int p, XArgs &a) {
  using MF = Mfma<T>;
  a.K = (p + 1) * (p + 1);
  m2l_table_layout<T>(p, a.KK, a.RP);
  a.nrt = a.RP / MF::TM;
  a.ngroups = (a.nrt + 3) / 4;
  a.nw = (a.nrt + a.ngroups - 1) / a.ngroups;
}

template <class T>
static size_t xlate_lds() {
  return (size_t)2 * XChunk<T>::KC * kBStride * sizeof(T);
}

// One wave per output row tile of a group, at least 3 waves (the gather
// uses 3 or 4 threads per target).  Blocks of exactly the active waves keep
// every SIMD of a CU busy with matrix-core work.
template <class T, int MODE, class... Args>
static void xlate_launch(const XArgs &a, int blocks, hipStream_t st, Args... args) {
  if (a.nw <= 3)
    hipLaunchKernelGGL((k_xlate<T, MODE, 3>), dim3(blocks), dim3(192), xlate_lds<T>(), st, args..., a);
  else
    hipLaunchKernelGGL((k_xlate<T, MODE, 4>), dim3(blocks), dim3(256), xlate_lds<T>(), st, args..., a);
}


template <class T>
void launch_xlate_m2l(const T *M, T *L, const T *Tab, const int4 *lists, int p, int KS, int d, int periodic, int lev_lo,
                      int lev_hi, hipStream_t st) {
  XArgs a;
  xlate_geometry<T>(p, a);
  a.KS = KS;
  a.d = std::min(d, lev_hi);
  a.periodic = periodic;
  a.lmin = std::max(periodic ? 1 : 2, lev_lo);
  a.nops = kListLen;
  a.level = 0;
  int blocks = 0;
  for (int l = 0; l <= 8; ++l) a.level_start[l] = 0;
  for (int l = a.lmin; l <= a.d; ++l) {
    a.level_start[l] = blocks;
    const int64_t np = int64_t(1) << (3 * (l - 1));
    blocks += (int)(8 * ((np + 63) / 64) * a.ngroups);
  }
  if (a.d + 1 <= 8) a.level_start[a.d + 1] = blocks;
  if (a.lmin > a.d || blocks == 0) return;
  xlate_launch<T, XL_M2L>(a, blocks, st, M, L, Tab, lists);
}

template <class T>
void launch_xlate_m2m(T *M, int lp, const T *Tab, const int4 *ops, int p, int KS, hipStream_t st) {
  XArgs a;
  xlate_geometry<T>(p, a);
  a.KS = KS;
  a.d = lp + 1;
  a.periodic = 0;
  a.lmin = 0;
  a.nops = 8;
  a.level = lp;
  const int64_t np = int64_t(1) << (3 * lp);
  const int blocks = (int)(((np + 63) / 64) * a.ngroups);
  xlate_launch<T, XL_M2M>(a, blocks, st, (const T *)M, M, Tab, ops);
}

template <class T>
void launch_xlate_l2l(T *L, int lc, const T *Tab, const int4 *ops, int p, int KS, hipStream_t st) {
  XArgs a;
  xlate_geometry<T>(p, a);
  a.KS = KS;
  a.d = lc;
  a.periodic = 0;
  a.lmin = 0;
  a.nops = 1;
  a.level = lc;
  const int64_t np = int64_t(1) << (3 * (lc - 1));
  const int blocks = (int)(8 * ((np + 63) / 64) * a.ngroups);
  xlate_launch<T, XL_L2L>(a, blocks, st, (const T *)L, L, Tab, ops);
}

// Operator stack for k_updown: A[c][k][r] = T_c[r][k] (r, k < K; zero padded to KS rows).
template <class T>
void updown_table(int K, int KS, const double *const *Tc, T *A) {
  for (int c = 0; c < 8; ++c)
    for (int k = 0; k < K; ++k)
      for (int r = 0; r < KS; ++r) A[((size_t)c * K + k) * KS + r] = r < K ? (T)Tc[c][(size_t)r * K + k] : T(0);
}

// parents per block: the largest of 8, 4, 2, 1 whose inputs (and, for M2M, child
// partials) fit in 64 KB of LDS
template <class T>
int updown_np(int KS, bool up) {
  int np = 8;
  while (np > 1 && (size_t)np * (up ? 16 : 1) * KS * sizeof(T) > 65536) np >>= 1;
  return np;
}

template <class T>
size_t updown_lds(int KS, bool up) {
  return (size_t)updown_np<T>(KS, up) * (up ? 16 : 1) * KS * sizeof(T);
}

template <class T, bool UP, int NP>
static void updown_go(T *X, const T *A, int K, int KS, int parent_level, hipStream_t st) {
  const int64_t nparent = int64_t(1) << (3 * parent_level);
  const int64_t blocks = (nparent + NP - 1) / NP;
  const int threads = std::min(1024, (8 * KS + 63) / 64 * 64);
  const size_t lds = (size_t)NP * (UP ? 16 : 1) * KS * sizeof(T);
  hipLaunchKernelGGL((k_updown<T, UP, NP>), dim3((unsigned)blocks), dim3(threads), lds, st, X, A, K, KS,
                     level_offset(parent_level), level_offset(parent_level + 1), nparent);
}

template <class T, bool UP>
static void updown_dispatch(T *X, const T *A, int K, int KS, int parent_level, hipStream_t st) {
  switch (updown_np<T>(KS, UP)) {
    case 8: updown_go<T, UP, 8>(X, A, K, KS, parent_level, st); break;
    case 4: updown_go<T, UP, 4>(X, A, K, KS, parent_level, st); break;
    case 2: updown_go<T, UP, 2>(X, A, K, KS, parent_level, st); break;
    default: updown_go<T, UP, 1>(X, A, K, KS, parent_level, st); break;
  }
}

template <class T>
void launch_updown(T *X, const T *A, int p, int KS, int parent_level, bool up, hipStream_t st) {
  const int K = (p + 1) * (p + 1);
  if (up) updown_dispatch<T, true>(X, A, K, KS, parent_level, st);
  else updown_dispatch<T, false>(X, A, K, KS, parent_level, st);
}

template <class T>
void launch_mfma_probe(const T *A, const T *B, T *C, int rows, int kk, hipStream_t st) {
  using MF = Mfma<T>;
  hipLaunchKernelGGL(k_mfma_probe<T>, dim3(1), dim3(64 * (rows / MF::TM)), 0, st, A, B, C, rows, kk);
}

void launch_mfma16_probe(const float *A, const float *B, float *C, int rows, int kk, hipStream_t st) {
  hipLaunchKernelGGL((k_mfma_probe<float, Mfma16f32>), dim3(1), dim3(64 * (rows / Mfma16f32::TM)), 0, st, A, B, C,
                     rows, kk);
}

template <class T>
int p2p_blocks(int d) {
  return 1 << (3 * d);  // one block per leaf
}

template <class T>
void launch_p2p(const Atom4<T> *sorted, const Atom4<T> *sorted_lo, const int *start, const int *perm, const T *Lleaf,
                int KS, const Geom *g, int d, int periodic, int p, double ke, T *phi_sorted, T *F, T *pot_user,
                double *epart, hipStream_t st, int mmax) {
  P2PArgs a;
  a.KS = KS;
  a.d = d;
  a.periodic = periodic;
  a.p = p;
  a.K = (p + 1) * (p + 1);
  a.ke = ke;
  a.mmax = mmax;
  // gradient coefficients in LDS when L, Dx, Dy, Dz fit in 16 KB
  a.dloc = (size_t)4 * a.K * sizeof(T) <= 16384 ? 1 : 0;
  const size_t lds = (size_t)(a.dloc ? 4 : 1) * a.K * sizeof(T);
  // without forces only the potential is formed (near field and local expansion);
  // with coordinate residuals (float32 above order 8) the pair displacements use them
  const dim3 grid(p2p_blocks<T>(d)), block(64);
  if (p == 8 && F)
    hipLaunchKernelGGL((k_p2p_l2p<T, 8, true, false>), grid, block, lds, st, sorted, sorted_lo, start, perm, Lleaf, g,
                       a, phi_sorted, F, pot_user, epart);
  else if (p == 8)
    hipLaunchKernelGGL((k_p2p_l2p<T, 8, false, false>), grid, block, lds, st, sorted, sorted_lo, start, perm, Lleaf, g,
                       a, phi_sorted, F, pot_user, epart);
  else if (F && sorted_lo)
    hipLaunchKernelGGL((k_p2p_l2p<T, 0, true, true>), grid, block, lds, st, sorted, sorted_lo, start, perm, Lleaf, g,
                       a, phi_sorted, F, pot_user, epart);
  else if (sorted_lo)
    hipLaunchKernelGGL((k_p2p_l2p<T, 0, false, true>), grid, block, lds, st, sorted, sorted_lo, start, perm, Lleaf, g,
                       a, phi_sorted, F, pot_user, epart);
  else if (F)
    hipLaunchKernelGGL((k_p2p_l2p<T, 0, true, false>), grid, block, lds, st, sorted, sorted_lo, start, perm, Lleaf, g,
                       a, phi_sorted, F, pot_user, epart);
  else
    hipLaunchKernelGGL((k_p2p_l2p<T, 0, false, false>), grid, block, lds, st, sorted, sorted_lo, start, perm, Lleaf, g,
                       a, phi_sorted, F, pot_user, epart);
}

template <class T>
void launch_charge_scale(const SiteArgs &s, const double *lam, T *qt, hipStream_t st) {
  if (s.n_sites == 0) return;
  hipLaunchKernelGGL(k_charge_scale<T>, dim3(s.n_sites), dim3(64), 0, st, s.atom_off, s.form_off, s.site_atoms, s.fq,
                     s.fq_off, lam, s.n_sites, qt);
}

// dynamic LDS of k_site: pair kernel, Rt, multipoles and lattice locals (with_d: plus the
// lattice locals' gradient coefficients)
size_t site_lds_bytes(int p, int maxa, int maxf, bool with_d) {
  const int K = (p + 1) * (p + 1);
  return sizeof(double) * (4 * (size_t)maxa * maxa + (size_t)maxa * K + (with_d ? 5 : 2) * (size_t)maxf * K);
}

bool site_in_lds(int p, int maxa, int maxf) {
  return site_lds_bytes(p, maxa, maxf, false) + kSiteStaticLds <= 65536;
}

template <class T>
void launch_site(const SiteArgs &s, const T *xyz, const int *slot_of, const Geom *g, const double *LamT,
                 const SiteIO<T> &io, hipStream_t st) {
  if (s.n_sites == 0) return;
  SiteArgs a = s;
  size_t lds = 0;
  if (io.ws) {
    a.dloc = 1;  // the workspace always has room for the gradient coefficients
  } else {
    // gradient coefficients in LDS when they fit next to the kernel's static arrays
    a.dloc = site_lds_bytes(s.p, s.maxa, s.maxf, true) + kSiteStaticLds <= 65536 ? 1 : 0;
    lds = site_lds_bytes(s.p, s.maxa, s.maxf, a.dloc != 0);
  }
  const dim3 grid(s.n_sites), block(256);
  if (s.p == 8 && io.ws)
    hipLaunchKernelGGL((k_site<T, 8, true>), grid, block, lds, st, a, xyz, slot_of, g, LamT, io);
  else if (s.p == 8)
    hipLaunchKernelGGL((k_site<T, 8, false>), grid, block, lds, st, a, xyz, slot_of, g, LamT, io);
  else if (io.ws)
    hipLaunchKernelGGL((k_site<T, 0, true>), grid, block, lds, st, a, xyz, slot_of, g, LamT, io);
  else
    hipLaunchKernelGGL((k_site<T, 0, false>), grid, block, lds, st, a, xyz, slot_of, g, LamT, io);
}

void launch_finalize(const double *epart, int nb, const double *dE_site, int ns, double ke, double *E, double *E_qi,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, epart, nb, dE_site, ns, ke, E, E_qi);
}


// One packed evaluation: octree build over the concatenated atoms and leaves
// (keys carry each system's first leaf, so one counting sort serves all),
// P2M, M2M by steps from each system's deepest level, M2L of every level of
// every system in one launch, the lattice per system, L2L by levels, near
// field, site correction and energy, all on stream st.
void launch_packed(const PackedPlan &pp, hipStream_t st) {
  const PackedSys *sys = pp.sys;
  const int ns = pp.nsys;
  hipLaunchKernelGGL(kp_bin, dim3(pp.atoms.blocks), dim3(256), 0, st, sys, pp.atoms.first, ns, pp.key, pp.rank,
                     pp.count, pp.packed);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, pp.count, pp.start, pp.nleaf);
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(pp.n_atoms, 256)), dim3(256), 0, st, pp.key, pp.rank, pp.start, pp.tmp,
                     pp.n_atoms);
  hipLaunchKernelGGL(k_leafsort<float>, dim3((pp.nleaf + 3) / 4), dim3(256), 0, st, pp.tmp, pp.start, pp.nleaf,
                     pp.packed, pp.perm, pp.slot_of, pp.sorted, nullptr, nullptr);
  const size_t p2m_lds = (size_t)pp.chunk * pp.K * sizeof(float);
  if (pp.p == 8)
    hipLaunchKernelGGL((kp_p2m<8>), dim3(pp.leaves.blocks), dim3(64), p2m_lds, st, sys, pp.leaves.first, ns,
                       pp.sorted, pp.start, pp.p, pp.K, pp.KS, pp.chunk, pp.Mc, pp.qds);
  else
    hipLaunchKernelGGL((kp_p2m<0>), dim3(pp.leaves.blocks), dim3(64), p2m_lds, st, sys, pp.leaves.first, ns,
                       pp.sorted, pp.start, pp.p, pp.K, pp.KS, pp.chunk, pp.Mc, pp.qds);
  const int np_up = updown_np<float>(pp.KS, true), np_dn = updown_np<float>(pp.KS, false);
  const int threads = std::min(1024, (8 * pp.KS + 63) / 64 * 64);
  auto updown = [&](bool up, int step, const PackedStage &stg) {
    if (stg.blocks == 0) return;
    const size_t lds = (size_t)(up ? np_up : np_dn) * (up ? 16 : 1) * pp.KS * sizeof(float);
    float *X = up ? pp.Mc : pp.Lc;
    const float *A = up ? pp.m2m : pp.l2l;
#define MAHI_KP_UPDOWN(U, N) \
  hipLaunchKernelGGL((kp_updown<U, N>), dim3(stg.blocks), dim3(threads), lds, st, sys, stg.first, ns, X, A, pp.K, pp.KS, step)
    if (up) {
      if (np_up == 8) MAHI_KP_UPDOWN(true, 8);
      else if (np_up == 4) MAHI_KP_UPDOWN(true, 4);
      else if (np_up == 2) MAHI_KP_UPDOWN(true, 2);
      else MAHI_KP_UPDOWN(true, 1);
    } else {
      if (np_dn == 8) MAHI_KP_UPDOWN(false, 8);
      else if (np_dn == 4) MAHI_KP_UPDOWN(false, 4);
      else if (np_dn == 2) MAHI_KP_UPDOWN(false, 2);
      else MAHI_KP_UPDOWN(false, 1);
    }
#undef MAHI_KP_UPDOWN
  };
  for (int j = 1; j <= pp.dmax; ++j) updown(true, j, pp.up[j - 1]);
  launch_packed_m2l(pp, st);
  hipLaunchKernelGGL(kp_lattice, dim3(ns), dim3(1024), 0, st, sys, pp.Mc, pp.Lc, pp.LamT, pp.K, pp.KS, pp.qds);
  for (int l = 1; l <= pp.dmax; ++l) updown(false, l, pp.down[l - 1]);
  const size_t p2p_lds = (size_t)4 * pp.K * sizeof(float) <= 16384 ? (size_t)4 * pp.K * sizeof(float)
                                                                     : (size_t)pp.K * sizeof(float);
  if (pp.p == 8)
    hipLaunchKernelGGL((kp_p2p<8>), dim3(pp.leaves.blocks), dim3(64), p2p_lds, st, sys, pp.leaves.first, ns,
                       pp.sorted, pp.start, pp.perm, pp.Lc, pp.KS, pp.phi_sorted, pp.epart);
  else
    hipLaunchKernelGGL((kp_p2p<0>), dim3(pp.leaves.blocks), dim3(64), p2p_lds, st, sys, pp.leaves.first, ns,
                       pp.sorted, pp.start, pp.perm, pp.Lc, pp.KS, pp.phi_sorted, pp.epart);
  if (pp.sites.blocks > 0) {
    if (pp.p == 8)
      hipLaunchKernelGGL((kp_site<8>), dim3(pp.sites.blocks), dim3(256), pp.site_lds, st, sys, pp.sites.first, ns,
                         pp.slot_of, pp.LamT);
    else
      hipLaunchKernelGGL((kp_site<0>), dim3(pp.sites.blocks), dim3(256), pp.site_lds, st, sys, pp.sites.first, ns,
                         pp.slot_of, pp.LamT);
  }
  hipLaunchKernelGGL(kp_finalize, dim3(ns), dim3(1024), 0, st, sys, pp.epart);
}

#define MAHI_INST(T)                                                                                                 \
  template void launch_bbox<T>(const T *, int64_t, double *, int, Geom *, hipStream_t);                             \
  template void launch_tree<T>(const T *, const T *, int64_t, const Geom *, int, int, TreeBufs<T>, hipStream_t);     \
  template void launch_p2m<T>(const Atom4<T> *, const int *, int, int, int, T *, double *, const Geom *, int,         \
                              hipStream_t);                                                                         \
  template void launch_lattice<T>(const T *, T *, const double *, int, const double *, Geom *, hipStream_t);            \
  template void m2l_table_layout<T>(int, int &, int &);                                                               \
  template void launch_mfma_probe<T>(const T *, const T *, T *, int, int, hipStream_t);                              \
  template void launch_xlate_m2l<T>(const T *, T *, const T *, const int4 *, int, int, int, int, int, int,            \
                                    hipStream_t);                                                                   \
  template void launch_xlate_m2m<T>(T *, int, const T *, const int4 *, int, int, hipStream_t);                        \
  template void launch_xlate_l2l<T>(T *, int, const T *, const int4 *, int, int, hipStream_t);                        \
  template void updown_table<T>(int, int, const double *const *, T *);                                               \
  template void launch_updown<T>(T *, const T *, int, int, int, bool, hipStream_t);                                   \
  template size_t updown_lds<T>(int, bool);                                                                           \
  template int updown_np<T>(int, bool);                                                                               \
  template int p2p_blocks<T>(int);                                                                                   \
  template void launch_p2p<T>(const Atom4<T> *, const Atom4<T> *, const int *, const int *, const T *, int,          \
                              const Geom *, int, int, int, double, T *, T *, T *, double *, hipStream_t, int);       \
  template void launch_charge_scale<T>(const SiteArgs &, const double *, T *, hipStream_t);                          \
  template void launch_site<T>(const SiteArgs &, const T *, const int *, const Geom *, const double *,               \
                               const SiteIO<T> &, hipStream_t);

MAHI_INST(float)
MAHI_INST(double)

}  // namespace mahi
