// Shared device-side definitions for the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mahi {

constexpr int kMaxOrder = 20;      // largest multipole order p supported
constexpr int kMaxSiteAtoms = 32;  // atoms per titratable site
constexpr int kMaxSiteForms = 16;  // forms per titratable site
constexpr int kListLen = 189;      // M2L interaction list length per parity class (well-separation 1)

// Root-cube geometry and the float64 charge moments that the periodic lattice
// needs; lives in device memory so that open boundaries can set it per call.
struct Geom {
  double origin[3];  // low corner of the root cube
  double edge;       // root cube edge
  double Q;          // sum of charges
  double D[3];       // sum q (x - c), c = root centre
  double S2;         // sum q |x - c|^2
};

template <class T>
struct alignas(4 * sizeof(T)) Atom4 {
  T x, y, z, q;  // position relative to the own leaf centre in leaf-edge units, and scaled charge
};

// 3-bit interleaved (Morton) box index; x is the most significant bit of each triple.
__host__ __device__ inline uint32_t spread3(uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) r |= ((v >> b) & 1u) << (3 * b);
  return r;
}
__host__ __device__ inline uint32_t compact3(uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) r |= ((v >> (3 * b)) & 1u) << b;
  return r;
}
__host__ __device__ inline uint32_t morton(uint32_t x, uint32_t y, uint32_t z) {
  return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}
__host__ __device__ inline void unmorton(uint32_t k, int &x, int &y, int &z) {
  x = (int)compact3(k >> 2);
  y = (int)compact3(k >> 1);
  z = (int)compact3(k);
}

// Number of boxes above level l (level offsets in the per-level coefficient arrays).
__host__ __device__ inline int64_t level_offset(int l) {
  int64_t o = 0, n = 1;
  for (int k = 0; k < l; ++k) {
    o += n;
    n *= 8;
  }
  return o;
}

// Periodic wrap into [0, L) in float64 (a result equal to L maps to 0).
__device__ inline double wrap_coord(double x, double L) {
  double w = x - L * floor(x / L);
  if (w >= L) w -= L;
  if (w < 0.0) w = 0.0;
  return w;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

}  // namespace mahi
