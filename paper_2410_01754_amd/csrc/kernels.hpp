// Host-visible launch functions of the gfx950 kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace mahi {

// float32 M2L: 128 targets per block, 96-row groups, k chunks of 80
// (a single 42-step chunk when (p+1)^2 = 81)
constexpr int kM2LKC = 80;
constexpr int kM2LTile = 128;
constexpr int kM2LRowGroup = 96;
constexpr int kM2LMaxSplit = 8;

struct M2LPlan {
  int K, KS, ns, nkc, ngroups, nsplit, ntiles;
  int nsplit_up;  // operator ranges of launches that end below level d - 1 (few tiles each)
  int tile0, tile_run;  // tiles of one launch (a level range)
  int d, lmin, periodic;
  int64_t nbox, zbox;  // boxes over all levels; index of the all-zero multipole row
  int tiles_start[9];
};

struct XArgs {
  int K, KS, KK, RP, nrt, nw, ngroups;
  int d, lmin, periodic, nops, level;
  int level_start[9];
};

struct P2PArgs {
  int d, periodic, p, K, KS, mmax, dloc;  // mmax: most targets per lane in a near-field pass (1..3)
  double ke;
};

// static LDS of the site kernel (per-site atom, form and result arrays), bytes
constexpr size_t kSiteStaticLds = 24576;

struct SiteArgs {
  int n_sites, p, K, periodic, maxa, maxf, dloc;
  double ke;
  const int *atom_off;    // [M+1] offsets into site_atoms
  const int *form_off;    // [M+1] offsets into the flat form list
  const int *fq_off;      // [M]   offsets into fq
  const int *site_atoms;  // [sum atoms]
  const double *fq;       // per site: form-major, atom-minor charges
  const double *lam;      // [sum forms]
};

// Inputs and outputs of the site correction.  The charge-scaled potential at a
// site atom comes from the tree (phi_sorted, leaf order, without ke) or, when
// pot_ext is set, from another solver (user order, scaled by ke).  F is
// accumulated at site atoms; every pointer except one potential may be null
// (dE_site is required).
template <class T>
struct SiteIO {
  const T *phi_sorted;
  const T *pot_ext;
  T *F;
  double *dvdl;     // [sum forms] ke (sum_i q^r_i V_i - C^r)
  double *dE_site;  // [M] intra-site correction energy (without ke)
  double *dedq;     // [sum forms * atoms] dE/dq^(s,r)_i, layout of the form charges
  double *dvdl_qi;  // [sum forms] ke sum_i q^r_i V_i (charge-interpolated derivative)
  double *ws;       // per-site work arrays in global memory when they exceed local memory
                    // (site s at ws + s * ws_stride doubles), else null
  int64_t ws_stride;
};

template <class T>
struct TreeBufs {
  int *key, *count, *start, *tmp, *perm, *slot_of;
  Atom4<T> *packed;  // leaf-local coordinates and scaled charge, input order
  Atom4<T> *sorted;  // the same, leaf order
  // float32 at orders above 8: the rounding residuals of the leaf-local
  // coordinates (x, y, z, 0), input and leaf order; null otherwise
  Atom4<T> *packed_lo = nullptr, *sorted_lo = nullptr;
};

// ---- packed batch: many periodic float32 systems of one order, every stage
// one launch over all of them (a block finds its system from its index).
// Offsets index the batch's concatenated arrays of atoms, leaves (8^d per
// system) and boxes (levels 0..d per system, then one all-zero row).
struct PackedSys {
  int64_t atom_off, n_atoms, box_off;
  int leaf_off, nleaf, d, n_sites;
  double ke;
  const float *xyz;  // the caller's positions [n_atoms][3] (device memory)
  const float *qt;   // scaled charges (the system's context)
  Geom *geom;        // the context's geometry; the lattice writes Q, D, S2 into it
  float *F;          // the caller's forces [n_atoms][3], or null
  float *pot;        // the caller's potential output [n_atoms], or null
  double *E;         // energy (the caller's, else the context's)
  double *E_qi;      // charge-interpolated energy, or null
  SiteArgs site;     // the context's site tables (maxa, maxf: the largest of the batch)
  SiteIO<float> io;  // site pass: the batch's potentials, F, dvdl, the context's dE_site
  M2LPlan plan;      // M2L items of the system over all its levels
  P2PArgs p2p;
};

// Block ranges of the per-system stages: system s owns blocks [first[s], first[s + 1]).
struct PackedStage {
  const int *first = nullptr;  // device [nsys + 1]
  int blocks = 0;
};

struct PackedPlan {
  const PackedSys *sys = nullptr;  // device [nsys]
  int nsys = 0, p = 8, K = 81, KS = 88, dmax = 0, nsplit = 1, nleaf = 0, chunk = 1;
  int64_t n_atoms = 0, nbox = 0;  // totals (nbox: boxes plus the zero row)
  size_t site_lds = 0;            // dynamic LDS of the site pass
  PackedStage atoms, leaves, m2l, sites, up[8], down[8];
  // batch buffers
  int *key, *rank, *count, *start, *tmp, *perm, *slot_of;
  Atom4<float> *packed, *sorted;
  float *phi_sorted, *Mc, *Lc, *part;
  double *qds, *epart;
  // tables shared by the systems (one order: identical tables)
  const float *m2l_tab, *m2m, *l2l;
  const int4 *lists;
  const double *LamT;
};

// One packed evaluation on stream st (every launch on that stream).
void launch_packed(const PackedPlan &pp, hipStream_t st);
void launch_packed_m2l(const PackedPlan &pp, hipStream_t st);

hipError_t upload_constants();
template <class T> void launch_bbox(const T *xyz, int64_t n, double *part, int nblk, Geom *g, hipStream_t st);
template <class T>
void launch_tree(const T *xyz, const T *qt, int64_t n, const Geom *g, int d, int periodic, TreeBufs<T> b, hipStream_t st);
template <class T>
void launch_p2m(const Atom4<T> *sorted, const int *start, int nleaf, int p, int KS, T *Mleaf, double *qds, const Geom *g,
                int d, hipStream_t st);
template <class T>
void launch_lattice(const T *M, T *L, const double *LamT, int K, const double *part, Geom *g, hipStream_t st);
// block partials of the lattice charge moments (kMomentBlocks rows of five)
constexpr int kMomentBlocks = 64;
void launch_moments(const double *qds, int nleaf, double *part, hipStream_t st);
template <class T> void m2l_table_layout(int p, int &KK, int &RP);
template <class T>
void launch_xlate_m2l(const T *M, T *L, const T *Tab, const int4 *lists, int p, int KS, int d, int periodic, int lev_lo,
                      int lev_hi, hipStream_t st);
template <class T> void launch_xlate_m2m(T *M, int lp, const T *Tab, const int4 *ops, int p, int KS, hipStream_t st);
template <class T> void launch_xlate_l2l(T *L, int lc, const T *Tab, const int4 *ops, int p, int KS, hipStream_t st);
void m2l32_plan(int p, int d, int periodic, int n_cu, M2LPlan &a);
void launch_m2l_f32(const float *M, float *L, float *part, const float *Tab, const int4 *lists, const M2LPlan &plan,
                    int lev_lo, int lev_hi, hipStream_t st);
void m2l32_table(const M2LPlan &a, int slot, const double *Tv, float *dst);
size_t m2l32_table_size(const M2LPlan &a, int nslots);
template <class T> void updown_table(int K, int KS, const double *const *Tc, T *A);
// float32 M2M/L2L on the matrix cores for orders up to 8 (rows of 88 floats)
size_t updown16_table_size(bool up);
void updown16_table(int K, const double *const *Tc, bool up, float *dst);
void launch_updown16(float *X, const float *A, int parent_level, bool up, hipStream_t st);
template <class T> size_t updown_lds(int KS, bool up);
template <class T> int updown_np(int KS, bool up);  // parents per block of k_updown
template <class T> void launch_updown(T *X, const T *A, int p, int KS, int parent_level, bool up, hipStream_t st);
template <class T> void launch_mfma_probe(const T *A, const T *B, T *C, int rows, int kk, hipStream_t st);
// the same check for the float32 16x16x4 tile of the M2L kernel for orders up to 8
void launch_mfma16_probe(const float *A, const float *B, float *C, int rows, int kk, hipStream_t st);
template <class T> int p2p_blocks(int d);
// sorted_lo: coordinate residuals (TreeBufs::sorted_lo) for the near field, or null
template <class T>
void launch_p2p(const Atom4<T> *sorted, const Atom4<T> *sorted_lo, const int *start, const int *perm, const T *Lleaf,
                int KS, const Geom *g, int d, int periodic, int p, double ke, T *phi_sorted, T *F, T *pot_user,
                double *epart, hipStream_t st, int mmax = 3);
template <class T> void launch_charge_scale(const SiteArgs &s, const double *lam, T *qt, hipStream_t st);
template <class T>
void launch_site(const SiteArgs &s, const T *xyz, const int *slot_of, const Geom *g, const double *LamT,
                 const SiteIO<T> &io, hipStream_t st);
void launch_finalize(const double *epart, int nb, const double *dE_site, int ns, double ke, double *E, double *E_qi,
                     hipStream_t st);
size_t site_lds_bytes(int p, int maxa, int maxf, bool with_d);
// Static device scratch of the allocation-free correction (mahi_correct_noalloc):
// its size, and its device address on `device` (looked up once per device with
// that device current; later calls return the kept address).
constexpr size_t kStaticScratchBytes = size_t(8) << 20;
hipError_t static_scratch(int device, void **ptr);
// whether the site pass keeps its work arrays in local memory (else a global workspace
// of site_lds_bytes(p, maxa, maxf, true) per site)
bool site_in_lds(int p, int maxa, int maxf);

}  // namespace mahi
