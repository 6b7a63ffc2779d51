// Float32 translations on the matrix cores (paper, section "Fast Multipole
// Method"): the multipole-to-local translation of the far field, for every
// box of levels 1..d (periodic) or 2..d (open) over its 189-box interaction
// list (kernels, the work decomposition M2LPlan and the operator table
// layout), and the upward and downward passes between the two deepest
// levels (M2M, L2L) for orders up to 8.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_common.hpp"
#include "kernels.hpp"

namespace mahi {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Source boxes by subtraction of dilated integers.  With a target's Morton
// index split into its x, y and z bits (t & mx, t & my, t & mz), the x bits of
// the index of box (x - dx) mod 2^l are ((t & mx) - dil(dx)) & mx: borrows run
// through the other axes' bit positions and are masked off, and the l-bit
// field wraps as the periodic lattice does.  The dilated offsets are the same
// for the whole wave (scalar work); a lane spends 3 subtractions, 3 masks and
// an OR per source instead of interleaving its coordinates.
__device__ __forceinline__ uint32_t dilate3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

struct AxisMasks {
  uint32_t x, y, z;
};

__device__ __forceinline__ AxisMasks axis_masks(int l) {
  const uint32_t mz = spread3((1u << l) - 1u);
  return {mz << 2, mz << 1, mz};
}

// Morton index (level-local) of the box at offset -v from the target whose
// index t has been split by the masks into tx, ty, tz.
__device__ __forceinline__ uint32_t dilated_source(const AxisMasks &m, uint32_t tx, uint32_t ty, uint32_t tz,
                                                   const int4 &v) {
  const uint32_t vx = (dilate3((uint32_t)v.x) << 2) & m.x;
  const uint32_t vy = (dilate3((uint32_t)v.y) << 1) & m.y;
  const uint32_t vz = dilate3((uint32_t)v.z) & m.z;
  return ((tx - vx) & m.x) | ((ty - vy) & m.y) | ((tz - vz) & m.z);
}

// ---------------------------------------------------------------------------
// M2L in float32 on the matrix cores, operator shared through LDS.
// Work item: (level, parity class, 128 consecutive targets of that class, row
// group of 96 output rows, range of operators of the 189-entry list).  A block
// has 4 waves; wave w owns 32 targets (one 32-column MFMA tile) and the 3 row
// tiles of the group.  For every (operator v, k chunk):
//   * the block stages T_v (96 rows x KC) once in LDS (double buffered);
//   * each wave holds its 32 gathered source multipoles in registers, loaded
//     as float4 from the padded multipole rows (stride KS, a multiple of 8);
//   * each wave runs 3 x NS MFMA 32x32x2 into 3 accumulator tiles.
// In k-step s the lanes of half h (lane >> 5) contract
//   k = 8 (s / 4) + 4 h + s % 4
// (the k index of one MFMA is internal to the instruction, so any pairing of
// the two halves works as long as A and B agree): each lane's B values are
// runs of 4 consecutive k, one float4 load per 4 steps.  The operator rows are
// stored pre-permuted (LDS row 2s + h holds that k); a chunk of NS = 40 steps
// covers 80 consecutive k.  Used for orders above 8 (k_m2l16_f32 serves the
// rest).  Several operator ranges of one target tile write separate partial
// sums that k_m2l_reduce adds in a fixed order.
// ---------------------------------------------------------------------------

template <int NS>
__device__ __forceinline__ void m2l32_body(const float *__restrict__ M, float *__restrict__ Out,
                                           const float *__restrict__ Tab, const int4 *__restrict__ lists,
                                           const M2LPlan &a, int bid) {
  constexpr int RG = kM2LRowGroup;  // rows per group (3 tiles of 32)
  constexpr int KC = 2 * NS;        // operator rows (k values) per chunk
  constexpr int NQ = (NS + 3) / 4;  // float4 loads per lane per chunk
  constexpr int AV = KC * RG / 4;   // float4 elements of one staged operator chunk
  constexpr int AR = (AV + 255) / 256;
  __shared__ float As[2][KC * RG];

  // ---- work item (blocks of one XCD take consecutive items)
  const int nitems = a.nsplit * a.ngroups * a.tile_run;
  const int item = (bid & 7) * (nitems >> 3) + (bid >> 3);
  const int tile = a.tile0 + item % a.tile_run;
  const int rest = item / a.tile_run;
  const int grp = rest % a.ngroups;
  const int split = rest / a.ngroups;
  int l = a.lmin;
  while (l < a.d && tile >= a.tiles_start[l + 1]) ++l;
  const int tl = tile - a.tiles_start[l];
  const int cls = tl & 7, chunk = tl >> 3;
  const int o0 = split * kListLen / a.nsplit, o1 = (split + 1) * kListLen / a.nsplit;
  const int nit = (o1 - o0) * a.nkc;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = lane >> 5, j = lane & 31;
  const int nl = 1 << l;
  const int64_t ntg = int64_t(1) << (3 * (l - 1));
  const int64_t P = (int64_t)chunk * kM2LTile + wave * 32 + j;
  const bool valid = P < ntg;
  // waves whose 32 targets are all empty (levels with few boxes) skip the matrix work
  const bool wave_busy = (int64_t)chunk * kM2LTile + wave * 32 < ntg;
  int tx = 0, ty = 0, tz = 0;
  if (valid) unmorton((uint32_t)(8 * P + cls), tx, ty, tz);
  const int64_t off = level_offset(l);
  const int4 *lst = lists + cls * kListLen;
  const AxisMasks am = axis_masks(l);
  const uint32_t tm = (uint32_t)(8 * P + cls);
  const uint32_t tmx = tm & am.x, tmy = tm & am.y, tmz = tm & am.z;

  // source row (in boxes) of operator iteration `it`, or the all-zero row
  auto src_row = [&](int it) -> int64_t {
    const int4 v = lst[o0 + it / a.nkc];
    bool ok = valid;
    if (!a.periodic)
      ok = ok && (unsigned)(tx - v.x) < (unsigned)nl && (unsigned)(ty - v.y) < (unsigned)nl &&
           (unsigned)(tz - v.z) < (unsigned)nl;
    return ok ? off + (int64_t)dilated_source(am, tmx, tmy, tmz, v) : a.zbox;
  };
  auto load_b = [&](int it, float *b) {
    const int c = it % a.nkc;
    const floatx4 *q = reinterpret_cast<const floatx4 *>(M + src_row(it) * a.KS + c * kM2LKC + 4 * h);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const floatx4 v = q[2 * i];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (4 * i + e < NS) b[4 * i + e] = v[e];
    }
  };
  auto a_src = [&](int it) {
    const int4 v = lst[o0 + it / a.nkc];
    const int c = it % a.nkc;
    return reinterpret_cast<const floatx4 *>(Tab + (((int64_t)v.w * a.ngroups + grp) * a.nkc + c) * (KC * RG));
  };
  auto load_a = [&](int it, floatx4 *r) {
    const floatx4 *q = a_src(it);
#pragma unroll
    for (int i = 0; i < AR; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < AV) r[i] = q[e];
    }
  };
  auto store_a = [&](int buf, const floatx4 *r) {
    floatx4 *dst = reinterpret_cast<floatx4 *>(As[buf]);
#pragma unroll
    for (int i = 0; i < AR; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < AV) dst[e] = r[i];
    }
  };

  floatx16 acc[3];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;

  float b0[NS], b1[NS];
  floatx4 ast[AR];
  load_a(0, ast);
  store_a(0, ast);
  load_a(min(1, nit - 1), ast);
  load_b(0, b0);
  __syncthreads();

  // one (operator, chunk) iteration: stage the next operator, prefetch the
  // next sources, then 3 x NS matrix-core steps on LDS buffer it & 1
  auto body = [&](int it, const float *bc, float *bn) {
    const int buf = it & 1;
    store_a(buf ^ 1, ast);
    load_a(min(it + 2, nit - 1), ast);
    load_b(min(it + 1, nit - 1), bn);
    const float *Ar = As[buf] + h * RG + j;
    if (wave_busy) {
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) {
#pragma unroll
        for (int t = 0; t < 3; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(Ar[2 * s2 * RG + 32 * t], bc[s2], acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  };
  for (int it = 0; it < nit; it += 2) {
    body(it, b0, b1);
    if (it + 1 < nit) body(it + 1, b1, b0);
  }

  // ---- results: lane (h, j) holds rows 8q + 4h + {0..3} of each row tile for target j
  if (!valid) return;
  const int64_t tb = off + 8 * P + cls;
  float *dst = Out + ((int64_t)split * a.nbox + tb) * a.KS;
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = grp * RG + 32 * t + 8 * q + 4 * h;
      if (row < a.KS) {
        floatx4 v;
        v[0] = acc[t][4 * q];
        v[1] = acc[t][4 * q + 1];
        v[2] = acc[t][4 * q + 2];
        v[3] = acc[t][4 * q + 3];
        *reinterpret_cast<floatx4 *>(dst + row) = v;
      }
    }
}

template <int NS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_m2l_f32(const float *__restrict__ M, float *__restrict__ Out, const float *__restrict__ Tab,
          const int4 *__restrict__ lists, M2LPlan a) {
  m2l32_body<NS>(M, Out, Tab, lists, a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// M2L in float32 for orders up to 8 ((p+1)^2 <= 81) on 16x16x4 matrix-core
// tiles.  The same work items, operator ranges, XCD mapping and LDS operator
// sharing as k_m2l_f32, but output rows 0..79 are 5 tiles of 16 and row 80 is
// formed on the vector ALU, so no matrix work is spent on padding rows.  Wave
// w owns targets 32w .. 32w+31 of the block as two 16-column halves; lane
// (q = lane / 16, c = lane % 16) supplies operator row c of a tile and the
// sources of targets c and c + 16.  In k-step s (21 per operator) lane group q
// contracts k = 20q + s (s < 20) or 80 + q (s = 20): each lane's sources are
// five float4 runs plus one shared float4.  The operator is stored in the
// order the lanes read it, so that one ds_read_b128 gives a lane the values of
// four consecutive k-steps of one row tile (8 MFMAs): steps 0..19 as
// [s / 4][q][t][c][s % 4], step 20 as [q][t][c], then the row-80 entries as
// [q][24 steps] (value A[k(s, q)][16 t + c] = T[16 t + c][k]).  The next group
// of four steps is read while the current one is multiplied.  Output tile
// registers: lane (q, c) holds rows 4q .. 4q+3 of its tile for its column.
// ---------------------------------------------------------------------------
template <int UNUSED>
struct M2L16 {
  static constexpr int NS = 21, RW = 80;
  static constexpr int TAIL = 5 * 4 * 5 * 16 * 4;  // steps 0..19: [g][q][t][c][4]  (6400)
  static constexpr int R80 = TAIL + 4 * 5 * 16;     // step 20: [q][t][c]            (6720)
  // row 80: [q][24 steps] at R80; zero padded to 7 float4 per thread of the
  // block, so that staging needs no bounds test: a guarded load splits the
  // loop into branches at which the compiler waits for every load in flight,
  // prefetches included
  static constexpr int AFL = 7 * 256 * 4;
  static constexpr int AV = AFL / 4;              // float4 per staged operator (1792)
  static constexpr int AR = (AV + 255) / 256;     // float4 per thread
};

// One piece of work: operators o0..o1-1 of the interaction list of one tile
// (128 targets of one parity class of one level); the partial locals go to
// slot `slot` of the output (Out + slot * nbox boxes).
__device__ __forceinline__ void m2l16_piece(const float *__restrict__ M, float *__restrict__ Out,
                                            const float *__restrict__ Tab, const int4 *__restrict__ lists,
                                            const M2LPlan &a, int tile, int o0, int o1, int slot) {
  using G = M2L16<0>;
  constexpr int NS = G::NS, AFL = G::AFL, AR = G::AR;
  __shared__ __attribute__((aligned(16))) float As[2][AFL];

  int l = a.lmin;
  while (l < a.d && tile >= a.tiles_start[l + 1]) ++l;
  const int tl = tile - a.tiles_start[l];
  const int cls = tl & 7, chunk = tl >> 3;
  const int nit = o1 - o0;
  const int split = slot;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane >> 4, c = lane & 15;
  const int nl = 1 << l;
  const int64_t ntg = int64_t(1) << (3 * (l - 1));
  const int64_t Pw = (int64_t)chunk * kM2LTile + wave * 32;
  // waves whose 32 targets are all empty (levels with few boxes) skip the matrix work
  const bool wave_busy = Pw < ntg;
  int64_t Ph[2];
  bool valid[2];
  int tx[2] = {0, 0}, ty[2] = {0, 0}, tz[2] = {0, 0};
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    Ph[hf] = Pw + 16 * hf + c;
    valid[hf] = Ph[hf] < ntg;
    if (valid[hf]) unmorton((uint32_t)(8 * Ph[hf] + cls), tx[hf], ty[hf], tz[hf]);
  }
  const int64_t off = level_offset(l);
  const int4 *lst = lists + cls * kListLen;
  const AxisMasks am = axis_masks(l);
  uint32_t tmx[2], tmy[2], tmz[2];
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    const uint32_t tm = (uint32_t)(8 * Ph[hf] + cls);
    tmx[hf] = tm & am.x;
    tmy[hf] = tm & am.y;
    tmz[hf] = tm & am.z;
  }

  // source row of target half hf for operator iteration it, or the all-zero row
  auto src_row = [&](int it, int hf) -> int64_t {
    const int4 v = lst[o0 + it];
    bool ok = valid[hf];
    if (!a.periodic)
      ok = ok && (unsigned)(tx[hf] - v.x) < (unsigned)nl && (unsigned)(ty[hf] - v.y) < (unsigned)nl &&
           (unsigned)(tz[hf] - v.z) < (unsigned)nl;
    return ok ? off + (int64_t)dilated_source(am, tmx[hf], tmy[hf], tmz[hf], v) : a.zbox;
  };
  // b[hf][s]: k = 20q + s (s < 20), 80 + q (s = 20)
  auto load_b = [&](int it, float (*b)[NS]) {
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      const float *row = M + src_row(it, hf) * a.KS;
      const floatx4 *qv = reinterpret_cast<const floatx4 *>(row + 20 * q);
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        const floatx4 v = qv[i];
        b[hf][4 * i + 0] = v[0];
        b[hf][4 * i + 1] = v[1];
        b[hf][4 * i + 2] = v[2];
        b[hf][4 * i + 3] = v[3];
      }
      b[hf][20] = row[80 + q];  // a per-lane address, not a select on loaded data (which would wait for it)
    }
  };
  auto a_src = [&](int it) {
    const int4 v = lst[o0 + it];
    return reinterpret_cast<const floatx4 *>(Tab + (int64_t)v.w * AFL);
  };
  auto load_a = [&](int it, floatx4 *r) {
    const floatx4 *src = a_src(it);
#pragma unroll
    for (int i = 0; i < AR; ++i) r[i] = src[threadIdx.x + 256 * i];
  };
  auto store_a = [&](int buf, const floatx4 *r) {
    floatx4 *dst = reinterpret_cast<floatx4 *>(As[buf]);
#pragma unroll
    for (int i = 0; i < AR; ++i) dst[threadIdx.x + 256 * i] = r[i];
  };

  floatx4 acc[5][2];
#pragma unroll
  for (int t = 0; t < 5; ++t)
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) acc[t][hf] = floatx4{0.f, 0.f, 0.f, 0.f};
  float r80[2] = {0.f, 0.f};

  float b0[2][NS], b1[2][NS];
  floatx4 ast[AR];
  load_a(0, ast);
  store_a(0, ast);
  load_a(min(1, nit - 1), ast);
  load_b(0, b0);
  __syncthreads();

  // one operator iteration: stage the next operator, prefetch the next
  // sources, then the matrix-core steps on LDS buffer it & 1
  auto body = [&](int it, float (*bc)[NS], float (*bn)[NS]) {
    const int buf = it & 1;
    store_a(buf ^ 1, ast);
    load_a(min(it + 2, nit - 1), ast);
    load_b(min(it + 1, nit - 1), bn);
    const floatx4 *A4 = reinterpret_cast<const floatx4 *>(As[buf]) + q * 80 + c;  // + (20 g + t) * 16
    const float *At = As[buf] + G::TAIL + q * 80 + c;                              // + 16 t
    const floatx4 *A80 = reinterpret_cast<const floatx4 *>(As[buf] + G::R80 + 24 * q);
    if (wave_busy) {
      floatx4 avn[5], a80n;
#pragma unroll
      for (int t = 0; t < 5; ++t) avn[t] = A4[t * 16];
      a80n = A80[0];
#pragma unroll
      for (int g = 0; g < 5; ++g) {
        floatx4 av[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) av[t] = avn[t];
        const floatx4 a80 = a80n;
        if (g < 4) {
#pragma unroll
          for (int t = 0; t < 5; ++t) avn[t] = A4[(20 * (g + 1) + t) * 16];
          a80n = A80[g + 1];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int s2 = 4 * g + j;
#pragma unroll
          for (int t = 0; t < 5; ++t)
#pragma unroll
            for (int hf = 0; hf < 2; ++hf)
              acc[t][hf] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t][j], bc[hf][s2], acc[t][hf], 0, 0, 0);
          r80[0] += a80[j] * bc[0][s2];
          r80[1] += a80[j] * bc[1][s2];
        }
      }
      float av[5];
#pragma unroll
      for (int t = 0; t < 5; ++t) av[t] = At[16 * t];
      const float a80 = As[buf][G::R80 + 24 * q + 20];
#pragma unroll
      for (int t = 0; t < 5; ++t)
#pragma unroll
        for (int hf = 0; hf < 2; ++hf)
          acc[t][hf] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], bc[hf][20], acc[t][hf], 0, 0, 0);
      r80[0] += a80 * bc[0][20];
      r80[1] += a80 * bc[1][20];
    }
    __syncthreads();
  };
  for (int it = 0; it < nit; it += 2) {
    body(it, b0, b1);
    if (it + 1 < nit) body(it + 1, b1, b0);
  }

  // row 80: sum the four k groups (lanes c, c + 16, c + 32, c + 48) in group order
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    const float v0 = __shfl(r80[hf], c, 64), v1 = __shfl(r80[hf], c + 16, 64);
    const float v2 = __shfl(r80[hf], c + 32, 64), v3 = __shfl(r80[hf], c + 48, 64);
    r80[hf] = ((v0 + v1) + v2) + v3;
  }
  // ---- results: rows 16t + 4q .. +3 for target 16 hf + c; row 80 and the zero pad by group 0
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    if (!valid[hf]) continue;
    const int64_t tb = off + 8 * Ph[hf] + cls;
    float *dst = Out + ((int64_t)split * a.nbox + tb) * a.KS;
#pragma unroll
    for (int t = 0; t < 5; ++t) *reinterpret_cast<floatx4 *>(dst + 16 * t + 4 * q) = acc[t][hf];
    if (q == 0) {
      *reinterpret_cast<floatx4 *>(dst + 80) = floatx4{r80[hf], 0.f, 0.f, 0.f};
      *reinterpret_cast<floatx4 *>(dst + 84) = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  }
}

// Block bid of the launch (a system of a batch passes its own block index):
// item = (tile, operator range), blocks of one XCD take consecutive items.
__device__ __forceinline__ void m2l16_body(const float *__restrict__ M, float *__restrict__ Out,
                                           const float *__restrict__ Tab, const int4 *__restrict__ lists,
                                           const M2LPlan &a, int bid) {
  const int nitems = a.nsplit * a.ngroups * a.tile_run;
  const int item = (bid & 7) * (nitems >> 3) + (bid >> 3);
  const int tile = a.tile0 + item % a.tile_run;
  const int split = item / a.tile_run;
  m2l16_piece(M, Out, Tab, lists, a, tile, split * kListLen / a.nsplit, (split + 1) * kListLen / a.nsplit, split);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_m2l16_f32(const float *__restrict__ M, float *__restrict__ Out, const float *__restrict__ Tab,
            const int4 *__restrict__ lists, M2LPlan a) {
  m2l16_body(M, Out, Tab, lists, a, blockIdx.x);
}

// Packed batch: the M2L items of every level of every system in one launch,
// writing operator-range partials into the batch's partial array.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
kp_m2l16(const PackedSys *__restrict__ sys, const int *__restrict__ first, int nsys, const float *__restrict__ Mc,
         float *__restrict__ part, const float *__restrict__ Tab, const int4 *__restrict__ lists, int KS) {
  int lo = 0, hi = nsys;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= (int)blockIdx.x) lo = mid;
    else hi = mid;
  }
  const PackedSys &S = sys[lo];
  m2l16_body(Mc + S.box_off * KS, part + S.box_off * KS, Tab, lists, S.plan, blockIdx.x - first[lo]);
}

// the same for orders above 8 (32x32x2 tiles, row groups of 96)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
kp_m2l32(const PackedSys *__restrict__ sys, const int *__restrict__ first, int nsys, const float *__restrict__ Mc,
         float *__restrict__ part, const float *__restrict__ Tab, const int4 *__restrict__ lists, int KS) {
  int lo = 0, hi = nsys;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= (int)blockIdx.x) lo = mid;
    else hi = mid;
  }
  const PackedSys &S = sys[lo];
  m2l32_body<40>(Mc + S.box_off * KS, part + S.box_off * KS, Tab, lists, S.plan, blockIdx.x - first[lo]);
}

// L[b] = sum over operator ranges s (in order) of the partial locals, for the
// boxes [b0, b1) of the M2L levels.
__global__ void k_m2l_reduce(const floatx4 *__restrict__ part, floatx4 *__restrict__ L, int64_t v0, int64_t v1,
                             int64_t stride, int nsplit) {
  for (int64_t i = v0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < v1; i += (int64_t)gridDim.x * blockDim.x) {
    floatx4 s = part[i];
    for (int k = 1; k < nsplit; ++k) s += part[i + k * stride];
    L[i] = s;
  }
}

// ---- float32 M2L plan: tiles of 128 targets, row groups of 96, operator ranges
void m2l32_plan(int p, int d, int periodic, int n_cu, M2LPlan &a) {
  a.K = (p + 1) * (p + 1);
  if (a.K <= 81) {
    // 16x16x4 kernel: one operator chunk of 21 steps (k <= 83), rows read up to k = 83
    a.ns = 21;
    a.nkc = 1;
    a.KS = 88;
  } else {
    a.ns = 40;
    a.nkc = (a.K + kM2LKC - 1) / kM2LKC;
    a.KS = a.nkc * kM2LKC;
  }
  a.ngroups = a.ns == 21 ? 1 : (a.K + kM2LRowGroup - 1) / kM2LRowGroup;
  a.d = d;
  a.periodic = periodic;
  a.lmin = periodic ? 1 : 2;
  a.nbox = level_offset(d + 1);
  a.zbox = a.nbox;
  a.ntiles = 0;
  for (int l = 0; l <= 8; ++l) a.tiles_start[l] = 0;
  for (int l = a.lmin; l <= d; ++l) {
    a.tiles_start[l] = a.ntiles;
    const int64_t ntg = int64_t(1) << (3 * (l - 1));
    a.ntiles += (int)(8 * ((ntg + kM2LTile - 1) / kM2LTile));
  }
  if (d + 1 <= 8) a.tiles_start[d + 1] = a.ntiles;
  a.tile0 = 0;
  a.tile_run = a.ntiles;
  // operator ranges: the split count minimising a fluid makespan model with
  // two resident blocks per CU, in units of one operator step of a block:
  //   max(work / slots + item / 2, item) + overhead * splits,
  // item = 189 nkc / s steps; the overhead (prologue of an item, partial
  // write and reduction) was fitted on the 1M-atom, depth-5 workload.
  a.nsplit = 1;
  if (a.ntiles > 0) {
    const double slots = 2.0 * (n_cu > 0 ? n_cu : 256);
    const double work = (double)a.ntiles * a.ngroups * kListLen * a.nkc;
    const double over = kListLen * a.nkc / 32.0;
    double best = 1e300;
    for (int s = 1; s <= kM2LMaxSplit; ++s) {
      const double item = (double)kListLen * a.nkc / s;
      const double cost = std::max(work / slots + 0.5 * item, item) + over * s;
      if (cost < best - 1e-9) {
        best = cost;
        a.nsplit = s;
      }
    }
  }
  // the upper levels hold a few tiles and run on a second stream beside the
  // main launch: their blocks are chains of operator steps, shortest with the
  // most ranges (measured: with 4 or 6 ranges that stream outlasts the main one)
  a.nsplit_up = kM2LMaxSplit;
}

void launch_m2l_f32(const float *M, float *L, float *part, const float *Tab, const int4 *lists, const M2LPlan &plan,
                    int lev_lo, int lev_hi, hipStream_t st) {
  lev_lo = std::max(lev_lo, plan.lmin);
  lev_hi = std::min(lev_hi, plan.d);
  if (plan.ntiles == 0 || lev_lo > lev_hi) return;
  M2LPlan a = plan;
  if (lev_hi < plan.d - 1) a.nsplit = plan.nsplit_up;
  a.tile0 = plan.tiles_start[lev_lo];
  a.tile_run = plan.tiles_start[lev_hi + 1] - a.tile0;  // a multiple of 8 (8 classes per chunk)
  if (a.tile_run <= 0) return;
  const int blocks = a.nsplit * a.ngroups * a.tile_run;
  float *out = a.nsplit > 1 ? part : L;
  if (a.ns == 21)
    hipLaunchKernelGGL(k_m2l16_f32, dim3(blocks), dim3(256), 0, st, M, out, Tab, lists, a);
  else
    hipLaunchKernelGGL(k_m2l_f32<40>, dim3(blocks), dim3(256), 0, st, M, out, Tab, lists, a);
  if (a.nsplit > 1) {
    const int64_t b0 = level_offset(lev_lo), b1 = level_offset(lev_hi + 1);
    const int64_t v0 = b0 * a.KS / 4, v1 = b1 * a.KS / 4;
    const int64_t n = v1 - v0;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_m2l_reduce, dim3(grid), dim3(256), 0, st, reinterpret_cast<const floatx4 *>(part),
                       reinterpret_cast<floatx4 *>(L), v0, v1, a.nbox * a.KS / 4, a.nsplit);
  }
}

void launch_packed_m2l(const PackedPlan &pp, hipStream_t st) {
  if (pp.m2l.blocks == 0) return;
  if (pp.K <= 81)
    hipLaunchKernelGGL(kp_m2l16, dim3(pp.m2l.blocks), dim3(256), 0, st, pp.sys, pp.m2l.first, pp.nsys, pp.Mc, pp.part,
                       pp.m2l_tab, pp.lists, pp.KS);
  else
    hipLaunchKernelGGL(kp_m2l32, dim3(pp.m2l.blocks), dim3(256), 0, st, pp.sys, pp.m2l.first, pp.nsys, pp.Mc, pp.part,
                       pp.m2l_tab, pp.lists, pp.KS);
  // every box of the batch: level-0 rows and the zero row hold all-zero partials
  const int64_t n = pp.nbox * pp.KS / 4;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_m2l_reduce, dim3(grid), dim3(256), 0, st, reinterpret_cast<const floatx4 *>(pp.part),
                     reinterpret_cast<floatx4 *>(pp.Lc), 0, n, n, pp.nsplit);
}

// Host layout of the float32 M2L operator table: [slot][row group][chunk][r][96]
// where LDS row r = 2s + h of a chunk holds k = 8(s/4) + 4h + s%4.
// ---------------------------------------------------------------------------
// M2M and L2L in float32 on the matrix cores, for orders up to 8 (K <= 81
// coefficients in rows padded to 88).  The children of parent P are the
// consecutive boxes 8P .. 8P+7, so both translations of a level are products
// with one operator stack:
//   M2M: M[P] (rows 0..87)        = sum_c T_c M[8P + c]
//   L2L: L[8P .. 8P+7] (704 rows) += S L[P],  S = the 8 operators S_c stacked
// A block of 4 waves takes 16 parents, the 16 columns of every 16x16x4 tile.
// Lane (q = lane / 16, c = lane % 16) holds parent c; in k-step s (21 per
// product) it contracts k = 20q + s (s < 20) or 80 + q (s = 20), so that its
// inputs are five float4 runs and one value, and pad rows of the inputs meet
// zero operator columns.  Operators are stored in the order the lanes read
// them: per 16-row tile, steps 0..19 as [s / 4][lane][s % 4] and step 20 as
// [lane], zero outside K x K.  Lane (q, c) ends with rows 4q .. 4q+3 of the
// tile for parent c.
//   M2M: wave w contracts children 2w and 2w + 1 into the 6 row tiles (rows
//   0..95, zero from K on); the four waves' tiles are added through LDS in
//   wave order and rows 0..87 written (pad rows as zeros).
//   L2L: wave w owns row tiles 11w .. 11w+10 of the 704 child rows and adds
//   them to the children in place (pad rows add zero).
// ---------------------------------------------------------------------------
constexpr int kUDRows = 88;          // padded coefficient rows of a box
constexpr int kUDTile = 21 * 64;     // floats of one operator tile in lane order
constexpr int kUDUpTiles = 6;        // M2M output rows 0..95
constexpr int kUDDnTiles = 44;       // L2L output rows: 8 children x 88
constexpr int kUDDnPerWave = 11;

__device__ __forceinline__ void ud_load_in(const float *__restrict__ src, int q, float *b) {
  const floatx4 *s4 = reinterpret_cast<const floatx4 *>(src + 20 * q);
#pragma unroll
  for (int g = 0; g < 5; ++g) {
    const floatx4 v = s4[g];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[4 * g + j] = v[j];
  }
  b[20] = q == 0 ? src[80] : 0.f;
}

struct UDTile {
  floatx4 a[5];
  float a20;
};

__device__ __forceinline__ void ud_load_tile(const float *__restrict__ tile, int lane, UDTile &r) {
  const floatx4 *a4 = reinterpret_cast<const floatx4 *>(tile) + lane;
#pragma unroll
  for (int g = 0; g < 5; ++g) r.a[g] = a4[64 * g];
  r.a20 = tile[1280 + lane];
}

__device__ __forceinline__ floatx4 ud_product(const UDTile &t, const float *b, floatx4 acc) {
#pragma unroll
  for (int g = 0; g < 5; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(t.a[g][j], b[4 * g + j], acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x4f32(t.a20, b[20], acc, 0, 0, 0);
}

__global__ void __launch_bounds__(256) k_m2m16(float *__restrict__ X, const float *__restrict__ A,
                                               int64_t off_parent, int64_t off_child, int64_t nparent) {
  __shared__ floatx4 red[4][kUDUpTiles][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int64_t P = (int64_t)blockIdx.x * 16 + c;
  const int64_t Pr = P < nparent ? P : 0;  // lanes past the last parent read parent 0 and write nothing
  floatx4 acc[kUDUpTiles];
#pragma unroll
  for (int t = 0; t < kUDUpTiles; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int ch = 2 * wave + h;
    float b[21];
    ud_load_in(X + (off_child + 8 * Pr + ch) * kUDRows, q, b);
    const float *At = A + (size_t)ch * kUDUpTiles * kUDTile;
    UDTile cur, nxt;
    ud_load_tile(At, lane, cur);
#pragma unroll
    for (int t = 0; t < kUDUpTiles; ++t) {
      if (t + 1 < kUDUpTiles) ud_load_tile(At + (t + 1) * kUDTile, lane, nxt);
      acc[t] = ud_product(cur, b, acc[t]);
      if (t + 1 < kUDUpTiles) cur = nxt;
    }
  }
#pragma unroll
  for (int t = 0; t < kUDUpTiles; ++t) red[wave][t][lane] = acc[t];
  __syncthreads();
  for (int e = threadIdx.x; e < kUDUpTiles * 64; e += 256) {
    const int t = e >> 6, l = e & 63;
    const int row = 16 * t + 4 * (l >> 4);
    const int64_t Pp = (int64_t)blockIdx.x * 16 + (l & 15);
    if (row < kUDRows && Pp < nparent) {
      floatx4 v = red[0][t][l];
      v += red[1][t][l];
      v += red[2][t][l];
      v += red[3][t][l];
      *reinterpret_cast<floatx4 *>(X + (off_parent + Pp) * kUDRows + row) = v;
    }
  }
}

__global__ void __launch_bounds__(256) k_l2l16(float *__restrict__ X, const float *__restrict__ A,
                                               int64_t off_parent, int64_t off_child, int64_t nparent) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int64_t P = (int64_t)blockIdx.x * 16 + c;
  const bool valid = P < nparent;
  float b[21];
  ud_load_in(X + (off_parent + (valid ? P : 0)) * kUDRows, q, b);
  float *dst = X + (off_child + 8 * (valid ? P : 0)) * kUDRows + 4 * q;
  const float *At = A + (size_t)wave * kUDDnPerWave * kUDTile;
  UDTile cur, nxt;
  ud_load_tile(At, lane, cur);
#pragma unroll
  for (int i = 0; i < kUDDnPerWave; ++i) {
    if (i + 1 < kUDDnPerWave) ud_load_tile(At + (i + 1) * kUDTile, lane, nxt);
    const floatx4 r = ud_product(cur, b, floatx4{0.f, 0.f, 0.f, 0.f});
    if (valid) {
      floatx4 *d4 = reinterpret_cast<floatx4 *>(dst + 16 * (kUDDnPerWave * wave + i));
      floatx4 v = *d4;
      v += r;
      *d4 = v;
    }
    if (i + 1 < kUDDnPerWave) cur = nxt;
  }
}

size_t updown16_table_size(bool up) { return (size_t)(up ? 8 * kUDUpTiles : kUDDnTiles) * kUDTile; }

// Lane-order stacks of k_m2m16 ([child][tile], T_c) and k_l2l16 ([tile], S_c
// of the child that owns the row); Tc[c] holds the K x K operator row-major.
void updown16_table(int K, const double *const *Tc, bool up, float *dst) {
  auto tile = [&](float *blk, auto elem) {
    for (int lane = 0; lane < 64; ++lane) {
      const int q = lane >> 4, c = lane & 15;
      for (int s = 0; s < 21; ++s) {
        const int k = s < 20 ? 20 * q + s : 80 + q;
        const float v = k < K ? elem(c, k) : 0.f;
        if (s < 20) blk[((s >> 2) * 64 + lane) * 4 + (s & 3)] = v;
        else blk[1280 + lane] = v;
      }
    }
  };
  if (up) {
    for (int ch = 0; ch < 8; ++ch)
      for (int t = 0; t < kUDUpTiles; ++t)
        tile(dst + (size_t)(ch * kUDUpTiles + t) * kUDTile, [&](int c, int k) {
          const int r = 16 * t + c;
          return r < K ? (float)Tc[ch][(size_t)r * K + k] : 0.f;
        });
  } else {
    for (int t = 0; t < kUDDnTiles; ++t)
      tile(dst + (size_t)t * kUDTile, [&](int c, int k) {
        const int R = 16 * t + c, ch = R / kUDRows, r = R % kUDRows;
        return r < K ? (float)Tc[ch][(size_t)r * K + k] : 0.f;
      });
  }
}

// parent_level: M2M writes that level from its children; L2L adds into the
// level below it.  X holds rows of 88 floats per box.
void launch_updown16(float *X, const float *A, int parent_level, bool up, hipStream_t st) {
  const int64_t nparent = int64_t(1) << (3 * parent_level);
  const dim3 grid((unsigned)((nparent + 15) / 16)), block(256);
  if (up)
    hipLaunchKernelGGL(k_m2m16, grid, block, 0, st, X, A, level_offset(parent_level), level_offset(parent_level + 1),
                       nparent);
  else
    hipLaunchKernelGGL(k_l2l16, grid, block, 0, st, X, A, level_offset(parent_level), level_offset(parent_level + 1),
                       nparent);
}

void m2l32_table(const M2LPlan &a, int slot, const double *Tv, float *dst) {
  if (a.ns == 21) {
    // k_m2l16_f32, per slot: steps 0..19 [s/4][q][t][c][s%4], step 20 [q][t][c], row 80 [q][24]
    using G = M2L16<0>;
    const int K = a.K;
    float *blk = dst + (size_t)slot * G::AFL;
    auto T = [&](int i, int k) { return (i < K && k < K) ? (float)Tv[(size_t)i * K + k] : 0.f; };
    for (int q = 0; q < 4; ++q)
      for (int t = 0; t < 5; ++t)
        for (int c = 0; c < 16; ++c) {
          for (int g = 0; g < 5; ++g)
            for (int j = 0; j < 4; ++j)
              blk[((((size_t)g * 4 + q) * 5 + t) * 16 + c) * 4 + j] = T(16 * t + c, 20 * q + 4 * g + j);
          blk[G::TAIL + ((size_t)q * 5 + t) * 16 + c] = T(16 * t + c, 80 + q);
        }
    for (int q = 0; q < 4; ++q)
      for (int s = 0; s < 24; ++s)
        blk[G::R80 + 24 * q + s] = s < 20 ? T(80, 20 * q + s) : (s == 20 ? T(80, 80 + q) : 0.f);
    return;
  }
  const int K = a.K, KC = 2 * a.ns;
  for (int g = 0; g < a.ngroups; ++g)
    for (int c = 0; c < a.nkc; ++c)
      for (int r = 0; r < KC; ++r) {
        const int s = r >> 1, h = r & 1;
        const int k = c * kM2LKC + 8 * (s >> 2) + 4 * h + (s & 3);
        float *row = dst + ((((size_t)slot * a.ngroups + g) * a.nkc + c) * KC + r) * kM2LRowGroup;
        for (int i = 0; i < kM2LRowGroup; ++i) {
          const int orow = g * kM2LRowGroup + i;
          row[i] = (orow < K && k < K) ? (float)Tv[(size_t)orow * K + k] : 0.f;
        }
      }
}

size_t m2l32_table_size(const M2LPlan &a, int nslots) {
  if (a.ns == 21) return (size_t)nslots * M2L16<0>::AFL;
  return (size_t)nslots * a.ngroups * a.nkc * (2 * a.ns) * kM2LRowGroup;
}

}  // namespace mahi
