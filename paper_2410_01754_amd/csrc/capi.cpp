// C ABI of libmahi.so (declared in include/mahi.h): validation, context
// lifecycle, table upload and the launch sequence of one evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/mahi.h"
#include "device_common.hpp"
#include "kernels.hpp"
#include "tables.hpp"

using namespace mahi;

namespace {

constexpr double kDefaultKe = 138.9354576;
constexpr int kSlots = 343;  // offsets v in [-3, 3]^3

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct mahi_ctx {
  int64_t N = 0;
  int periodic = 1;
  double edge = 0.0;
  int p = 8, d = 0, prec = 32;
  int KS = 0;      // stride of one box's coefficients in the multipole/local arrays (>= (p+1)^2, zero padded)
  int n_cu = 256;  // compute units of the device
  M2LPlan plan32{};  // float32 M2L decomposition
  int p2p_mmax = 3;  // most near-field targets per lane (mahi_tune may lower it)
  double ke = kDefaultKe;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int M = 0, nforms = 0, nsite_atoms = 0, maxa = 0, maxf = 0;
  int64_t nfq = 0;  // form charges over all sites
  bool lambda_set = false;
  std::string err;
  std::vector<DevBuf> bufs;

  // device buffers (element type T = float or double for the FMM arrays)
  void *xyz = nullptr, *qt = nullptr, *F = nullptr, *pot = nullptr, *phi_sorted = nullptr;
  void *part = nullptr;  // float32 M2L partial locals, one array per operator range
  void *packed = nullptr;  // leaf-local atoms in input order (octree build)
  void *packed_lo = nullptr, *sorted_lo = nullptr;  // float32 above order 8: coordinate residuals
  void *Mc = nullptr, *Lc = nullptr, *m2l = nullptr, *m2m = nullptr, *l2l = nullptr, *sorted = nullptr;
  void *m2m16 = nullptr, *l2l16 = nullptr;  // float32, orders up to 8: matrix-core M2M/L2L operator stacks
  double *LamT = nullptr, *qds = nullptr, *epart = nullptr, *dE_site = nullptr, *dvdl = nullptr, *E = nullptr;
  double *bbox = nullptr, *lam = nullptr, *fq = nullptr;
  double *dedq = nullptr, *dvdl_qi = nullptr, *E_qi = nullptr;  // host-I/O staging of the optional outputs
  double *site_ws = nullptr;  // site-pass work arrays in global memory when they exceed local memory
  int64_t site_ws_stride = 0;  // doubles per site
  int4 *lists = nullptr;
  Geom *geom = nullptr;
  int *key = nullptr, *count = nullptr, *start = nullptr, *tmp = nullptr, *perm = nullptr,
      *slot_of = nullptr;
  int *atom_off = nullptr, *form_off = nullptr, *fq_off = nullptr, *site_atoms = nullptr;
  int nbbox = 256;
  // second stream (default priority) for the upper tree levels (M2M above the two
  // deepest levels, the periodic lattice, their M2L and L2L), beside the main
  // M2L; fork/join events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // stage profiling: events[eval][slot]; slots 0..MAHI_N_STAGES are the stage
  // boundaries on the main stream, the last two bracket the upper levels on the side stream
  static constexpr int kSlots = MAHI_N_STAGES + 3;
  std::vector<hipEvent_t> prof_events;
  int prof_max = 0, prof_n = 0;
  std::vector<double> prof_totals;  // per-evaluation durations of the last ended profile
  bool prof_done = false;
  void mark(int boundary) {
    if (prof_n < prof_max) (void)hipEventRecord(prof_events[(size_t)prof_n * kSlots + boundary], stream);
  }
  void mark_side(int which) {
    if (prof_n < prof_max) (void)hipEventRecord(prof_events[(size_t)prof_n * kSlots + MAHI_N_STAGES + 1 + which], side);
  }

  mahi_status fail(mahi_status s, const std::string &m) {
    err = m;
    return s;
  }
  template <class P>
  hipError_t alloc(P *&ptr, size_t bytes) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes < 16 ? 16 : bytes);
    if (e != hipSuccess) return e;
    bufs.push_back({q, bytes});
    ptr = static_cast<P *>(q);
    return hipSuccess;
  }
};

struct mahi_batch {
  std::vector<mahi_ctx *> ctxs;
  int device = 0;
  bool use_graph = false;
  hipStream_t root = nullptr;
  bool own_root = false;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<mahi_eval_args> captured;  // the arguments baked into the graph
  // packed mode: every stage one launch over all systems, on `root` only
  bool packed = false;
  PackedPlan pp{};
  std::vector<DevBuf> bufs;           // the batch's own device memory
  std::vector<PackedSys> sys_host;    // per-system descriptors (argument pointers filled per call)
  PackedSys *sys_dev = nullptr;
  std::vector<mahi_eval_args> table;  // the arguments the device descriptors hold
  std::string err;
  mahi_status fail(mahi_status s, const std::string &m) {
    err = m;
    return s;
  }
  template <class P>
  hipError_t alloc(P *&ptr, size_t bytes) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes < 16 ? 16 : bytes);
    if (e != hipSuccess) return e;
    bufs.push_back({q, bytes});
    ptr = static_cast<P *>(q);
    return hipSuccess;
  }
};

namespace {

thread_local std::string g_create_error;

bool is_fin(double v) { return std::isfinite(v); }

template <class T>
void to_layout_transposed(int K, const std::vector<double> &rowmajor, T *out) {
  // out[c][r] = T[r][c]
  for (int r = 0; r < K; ++r)
    for (int c = 0; c < K; ++c) out[(size_t)c * K + r] = (T)rowmajor[(size_t)r * K + c];
}

// The 8 parity-class interaction lists: target child c of parent P; sources are
// the children of P's 27 neighbours that are not adjacent to the target.
std::vector<int4> class_lists() {
  std::vector<int4> out;
  for (int c = 0; c < 8; ++c) {
    const int cx = (c >> 2) & 1, cy = (c >> 1) & 1, cz = c & 1;
    int cnt = 0;
    for (int px = -1; px <= 1; ++px)
      for (int py = -1; py <= 1; ++py)
        for (int pz = -1; pz <= 1; ++pz)
          for (int s = 0; s < 8; ++s) {
            const int sx = (s >> 2) & 1, sy = (s >> 1) & 1, sz = s & 1;
            const int vx = cx - (2 * px + sx), vy = cy - (2 * py + sy), vz = cz - (2 * pz + sz);
            if (std::max(std::abs(vx), std::max(std::abs(vy), std::abs(vz))) <= 1) continue;
            int4 e;
            e.x = vx;
            e.y = vy;
            e.z = vz;
            e.w = (vx + 3) * 49 + (vy + 3) * 7 + (vz + 3);
            out.push_back(e);
            ++cnt;
          }
    (void)cnt;
  }
  return out;
}

const char *hip_msg(hipError_t e) { return hipGetErrorString(e); }

#define HIP_TRY(expr, what)                                                                 \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess) return ctx->fail(MAHI_EDEVICE, std::string(what) + ": " + hip_msg(_e)); \
  } while (0)

template <class T>
mahi_status setup_device(mahi_ctx *ctx, const std::vector<double> &q_env, const std::vector<int> &atom_off,
                         const std::vector<int> &form_off, const std::vector<int> &fq_off,
                         const std::vector<int> &site_atoms, const std::vector<double> &fq) {
  const int p = ctx->p, d = ctx->d, K = ncoef(p);
  const int64_t N = ctx->N;
  const int nleaf = 1 << (3 * d);
  const int64_t nbox = level_offset(d + 1);
  const bool f32 = sizeof(T) == sizeof(float);
  if (f32) {
    m2l32_plan(p, d, ctx->periodic, ctx->n_cu, ctx->plan32);
    ctx->KS = ctx->plan32.KS;
  } else {
    ctx->KS = K;
  }
  const int KS = ctx->KS;
  HIP_TRY(upload_constants(), "constant tables");
  HIP_TRY(ctx->alloc(ctx->xyz, sizeof(T) * 3 * N), "alloc xyz");
  HIP_TRY(ctx->alloc(ctx->qt, sizeof(T) * N), "alloc charges");
  HIP_TRY(ctx->alloc(ctx->F, sizeof(T) * 3 * N), "alloc forces");
  HIP_TRY(ctx->alloc(ctx->pot, sizeof(T) * N), "alloc potential");
  HIP_TRY(ctx->alloc(ctx->phi_sorted, sizeof(T) * N), "alloc potential (sorted)");
  HIP_TRY(ctx->alloc(ctx->sorted, sizeof(Atom4<T>) * N), "alloc sorted atoms");
  HIP_TRY(ctx->alloc(ctx->packed, sizeof(Atom4<T>) * N), "alloc packed atoms");
  if (f32 && p > 8) {
    HIP_TRY(ctx->alloc(ctx->packed_lo, sizeof(Atom4<T>) * N), "alloc coordinate residuals");
    HIP_TRY(ctx->alloc(ctx->sorted_lo, sizeof(Atom4<T>) * N), "alloc coordinate residuals");
  }
  // one extra all-zero box row (the source of empty M2L slots); pads stay zero
  HIP_TRY(ctx->alloc(ctx->Mc, sizeof(T) * (nbox + 1) * KS), "alloc multipoles");
  HIP_TRY(ctx->alloc(ctx->Lc, sizeof(T) * (nbox + 1) * KS), "alloc locals");
  HIP_TRY(hipMemset(ctx->Mc, 0, sizeof(T) * (nbox + 1) * KS), "zero multipoles");
  HIP_TRY(hipMemset(ctx->Lc, 0, sizeof(T) * (nbox + 1) * KS), "zero locals");
  const int nsplit_max = f32 ? std::max(ctx->plan32.nsplit, ctx->plan32.nsplit_up) : 1;
  if (nsplit_max > 1) HIP_TRY(ctx->alloc(ctx->part, sizeof(T) * nsplit_max * nbox * KS), "alloc M2L partials");
  HIP_TRY(ctx->alloc(ctx->key, sizeof(int) * N), "alloc keys");
  HIP_TRY(ctx->alloc(ctx->tmp, sizeof(int) * N), "alloc scatter");
  HIP_TRY(ctx->alloc(ctx->perm, sizeof(int) * N), "alloc perm");
  HIP_TRY(ctx->alloc(ctx->slot_of, sizeof(int) * N), "alloc slot map");
  HIP_TRY(ctx->alloc(ctx->count, sizeof(int) * nleaf), "alloc counts");
  HIP_TRY(hipMemset(ctx->count, 0, sizeof(int) * nleaf), "zero counts");  // k_scan clears them after each use
  HIP_TRY(ctx->alloc(ctx->start, sizeof(int) * (nleaf + 1)), "alloc starts");
  HIP_TRY(ctx->alloc(ctx->qds, sizeof(double) * 5 * (nleaf + kMomentBlocks)), "alloc moments");  // + block partials
  HIP_TRY(ctx->alloc(ctx->epart, sizeof(double) * p2p_blocks<T>(d)), "alloc energy partials");
  HIP_TRY(ctx->alloc(ctx->E, sizeof(double) * 1), "alloc energy");
  HIP_TRY(ctx->alloc(ctx->E_qi, sizeof(double) * 1), "alloc energy");
  HIP_TRY(ctx->alloc(ctx->bbox, sizeof(double) * 6 * ctx->nbbox), "alloc bbox");
  HIP_TRY(ctx->alloc(ctx->geom, sizeof(Geom)), "alloc geometry");
  HIP_TRY(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking), "side stream");
  HIP_TRY(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming), "event create");
  HIP_TRY(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming), "event create");
  Geom g{};
  g.edge = ctx->periodic ? ctx->edge : 1.0;
  HIP_TRY(hipMemcpy(ctx->geom, &g, sizeof(Geom), hipMemcpyHostToDevice), "upload geometry");
  {
    std::vector<T> qh(N);
    for (int64_t i = 0; i < N; ++i) qh[i] = (T)q_env[i];
    HIP_TRY(hipMemcpy(ctx->qt, qh.data(), sizeof(T) * N, hipMemcpyHostToDevice), "upload charges");
  }
  // M2L table layout of k_xlate (float64): [op][k (padded)][row (padded)]
  int KK, RP;
  m2l_table_layout<T>(p, KK, RP);
  {
    // child c of a parent sits at offset delta_c (parent units); stacks A[c][k][r] for k_updown
    std::vector<std::vector<double>> Tup(8, std::vector<double>((size_t)K * K)), Tdn(8, std::vector<double>((size_t)K * K));
    const double *pu[8], *pd[8];
    for (int s = 0; s < 8; ++s) {
      const double delta[3] = {(((s >> 2) & 1) - 0.5) * 0.5, (((s >> 1) & 1) - 0.5) * 0.5, ((s & 1) - 0.5) * 0.5};
      m2m_matrix(p, delta, Tup[s].data());
      l2l_matrix(p, delta, Tdn[s].data());
      pu[s] = Tup[s].data();
      pd[s] = Tdn[s].data();
    }
    std::vector<T> up((size_t)8 * K * KS), dn((size_t)8 * K * KS);
    updown_table<T>(K, KS, pu, up.data());
    updown_table<T>(K, KS, pd, dn.data());
    HIP_TRY(ctx->alloc(ctx->m2m, sizeof(T) * up.size()), "alloc m2m");
    HIP_TRY(ctx->alloc(ctx->l2l, sizeof(T) * dn.size()), "alloc l2l");
    HIP_TRY(hipMemcpy(ctx->m2m, up.data(), sizeof(T) * up.size(), hipMemcpyHostToDevice), "upload m2m");
    HIP_TRY(hipMemcpy(ctx->l2l, dn.data(), sizeof(T) * dn.size(), hipMemcpyHostToDevice), "upload l2l");
    if (f32 && K <= 81 && KS == 88) {
      std::vector<float> up16(updown16_table_size(true)), dn16(updown16_table_size(false));
      updown16_table(K, pu, true, up16.data());
      updown16_table(K, pd, false, dn16.data());
      HIP_TRY(ctx->alloc(ctx->m2m16, sizeof(float) * up16.size()), "alloc m2m");
      HIP_TRY(ctx->alloc(ctx->l2l16, sizeof(float) * dn16.size()), "alloc l2l");
      HIP_TRY(hipMemcpy(ctx->m2m16, up16.data(), sizeof(float) * up16.size(), hipMemcpyHostToDevice), "upload m2m");
      HIP_TRY(hipMemcpy(ctx->l2l16, dn16.data(), sizeof(float) * dn16.size(), hipMemcpyHostToDevice), "upload l2l");
    }
  }
  const int lmin = ctx->periodic ? 1 : 2;
  if (d >= lmin) {
    // float32: operator-shared layout of k_m2l_f32; float64: [slot][k][row] of k_xlate
    std::vector<T> tab(f32 ? m2l32_table_size(ctx->plan32, kSlots) : (size_t)kSlots * KK * RP, T(0));
    std::vector<double> Tv((size_t)K * K);
    for (int slot = 0; slot < kSlots; ++slot) {
      const int vx = slot / 49 - 3, vy = (slot / 7) % 7 - 3, vz = slot % 7 - 3;
      if (std::max(std::abs(vx), std::max(std::abs(vy), std::abs(vz))) <= 1) continue;
      const double v[3] = {double(vx), double(vy), double(vz)};
      m2l_matrix(p, v, Tv.data());
      if (f32) {
        m2l32_table(ctx->plan32, slot, Tv.data(), reinterpret_cast<float *>(tab.data()));
        continue;
      }
      T *dst = tab.data() + (size_t)slot * KK * RP;
      for (int r = 0; r < K; ++r)
        for (int c = 0; c < K; ++c) dst[(size_t)c * RP + r] = (T)Tv[(size_t)r * K + c];
    }
    HIP_TRY(ctx->alloc(ctx->m2l, sizeof(T) * tab.size()), "alloc m2l table");
    HIP_TRY(hipMemcpy(ctx->m2l, tab.data(), sizeof(T) * tab.size(), hipMemcpyHostToDevice), "upload m2l table");
    std::vector<int4> lists = class_lists();
    HIP_TRY(ctx->alloc(ctx->lists, sizeof(int4) * lists.size()), "alloc lists");
    HIP_TRY(hipMemcpy(ctx->lists, lists.data(), sizeof(int4) * lists.size(), hipMemcpyHostToDevice), "upload lists");
  }
  {
    std::vector<double> Lam((size_t)K * K, 0.0), LamT((size_t)K * K, 0.0);
    if (ctx->periodic) lattice_matrix(p, Lam.data());
    for (int r = 0; r < K; ++r)
      for (int c = 0; c < K; ++c) LamT[(size_t)c * K + r] = Lam[(size_t)r * K + c];
    HIP_TRY(ctx->alloc(ctx->LamT, sizeof(double) * LamT.size()), "alloc lattice");
    HIP_TRY(hipMemcpy(ctx->LamT, LamT.data(), sizeof(double) * LamT.size(), hipMemcpyHostToDevice), "upload lattice");
  }
  // sites
  if (ctx->M > 0) {
    HIP_TRY(ctx->alloc(ctx->atom_off, sizeof(int) * atom_off.size()), "alloc sites");
    HIP_TRY(ctx->alloc(ctx->form_off, sizeof(int) * form_off.size()), "alloc sites");
    HIP_TRY(ctx->alloc(ctx->fq_off, sizeof(int) * fq_off.size()), "alloc sites");
    HIP_TRY(ctx->alloc(ctx->site_atoms, sizeof(int) * site_atoms.size()), "alloc sites");
    HIP_TRY(ctx->alloc(ctx->fq, sizeof(double) * fq.size()), "alloc sites");
    HIP_TRY(ctx->alloc(ctx->lam, sizeof(double) * ctx->nforms), "alloc lambda");
    HIP_TRY(ctx->alloc(ctx->dvdl, sizeof(double) * ctx->nforms), "alloc dvdl");
    HIP_TRY(ctx->alloc(ctx->dvdl_qi, sizeof(double) * ctx->nforms), "alloc dvdl");
    HIP_TRY(ctx->alloc(ctx->dedq, sizeof(double) * fq.size()), "alloc dE/dq");
    if (!site_in_lds(p, ctx->maxa, ctx->maxf)) {
      ctx->site_ws_stride = (int64_t)(site_lds_bytes(p, ctx->maxa, ctx->maxf, true) / sizeof(double));
      HIP_TRY(ctx->alloc(ctx->site_ws, sizeof(double) * ctx->site_ws_stride * ctx->M), "alloc site workspace");
    }
    HIP_TRY(ctx->alloc(ctx->dE_site, sizeof(double) * ctx->M), "alloc site energies");
    HIP_TRY(hipMemcpy(ctx->atom_off, atom_off.data(), sizeof(int) * atom_off.size(), hipMemcpyHostToDevice), "upload");
    HIP_TRY(hipMemcpy(ctx->form_off, form_off.data(), sizeof(int) * form_off.size(), hipMemcpyHostToDevice), "upload");
    HIP_TRY(hipMemcpy(ctx->fq_off, fq_off.data(), sizeof(int) * fq_off.size(), hipMemcpyHostToDevice), "upload");
    HIP_TRY(hipMemcpy(ctx->site_atoms, site_atoms.data(), sizeof(int) * site_atoms.size(), hipMemcpyHostToDevice),
            "upload");
    HIP_TRY(hipMemcpy(ctx->fq, fq.data(), sizeof(double) * fq.size(), hipMemcpyHostToDevice), "upload");
  }
  return MAHI_OK;
}

template <class T>
SiteArgs site_args(const mahi_ctx *ctx) {
  SiteArgs s;
  s.n_sites = ctx->M;
  s.p = ctx->p;
  s.K = ncoef(ctx->p);
  s.periodic = ctx->periodic;
  s.maxa = ctx->maxa;
  s.maxf = ctx->maxf;
  s.ke = ctx->ke;
  s.atom_off = ctx->atom_off;
  s.form_off = ctx->form_off;
  s.fq_off = ctx->fq_off;
  s.site_atoms = ctx->site_atoms;
  s.fq = ctx->fq;
  s.lam = ctx->lam;
  return s;
}

template <class T>
mahi_status eval_impl(mahi_ctx *ctx, const mahi_eval_args *a) {
  const bool dev = (a->flags & MAHI_DEVICE_IO) != 0;
  const int64_t N = ctx->N;
  const int p = ctx->p, d = ctx->d, KS = ctx->KS, nleaf = 1 << (3 * d);
  hipStream_t st = ctx->stream;
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  const T *xyz = static_cast<const T *>(a->xyz);
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(ctx->xyz, a->xyz, sizeof(T) * 3 * N, hipMemcpyHostToDevice, st), "copy positions");
    xyz = static_cast<const T *>(ctx->xyz);
  }
  T *F = dev ? static_cast<T *>(a->forces) : (a->forces ? static_cast<T *>(ctx->F) : nullptr);
  T *pot = dev ? static_cast<T *>(a->potential) : (a->potential ? static_cast<T *>(ctx->pot) : nullptr);
  double *E = (dev && a->energy) ? a->energy : ctx->E;
  double *dvdl = (dev && a->dvdl) ? a->dvdl : ctx->dvdl;
  if (ctx->M > 0 && !dvdl) dvdl = ctx->dvdl;
  double *dedq = (ctx->M > 0 && a->dedq) ? (dev ? a->dedq : ctx->dedq) : nullptr;
  double *dvdl_qi = (ctx->M > 0 && a->dvdl_qi) ? (dev ? a->dvdl_qi : ctx->dvdl_qi) : nullptr;
  double *E_qi = a->energy_qi ? (dev ? a->energy_qi : ctx->E_qi) : nullptr;

  T *Mc = static_cast<T *>(ctx->Mc), *Lc = static_cast<T *>(ctx->Lc);
  ctx->mark(0);
  if (!ctx->periodic) launch_bbox<T>(xyz, N, ctx->bbox, ctx->nbbox, ctx->geom, st);
  TreeBufs<T> tb{ctx->key,     ctx->count,   ctx->start, ctx->tmp, ctx->perm, ctx->slot_of,
                 static_cast<Atom4<T> *>(ctx->packed), static_cast<Atom4<T> *>(ctx->sorted),
                 static_cast<Atom4<T> *>(ctx->packed_lo), static_cast<Atom4<T> *>(ctx->sorted_lo)};
  launch_tree<T>(xyz, static_cast<const T *>(ctx->qt), N, ctx->geom, d, ctx->periodic, tb, st);
  ctx->mark(1);
  launch_p2m<T>(tb.sorted, ctx->start, nleaf, p, KS, Mc + level_offset(d) * KS, ctx->periodic ? ctx->qds : nullptr,
                ctx->geom, d, st);
  ctx->mark(2);
  // Levels hl..d (hl = max(lmin, d - 1)) carry almost all M2L work, and need
  // multipoles of levels d - 1 and d only.  After the M2M into level d - 1 the
  // side stream takes the lattice charge moments, the M2M into levels
  // d - 2..0, M2L of levels lmin..hl-1 (issued before the main launch, so its
  // blocks are dispatched beside it), the periodic lattice and L2L into
  // levels up to hl - 1, while the main
  // stream runs M2L of levels hl..d.  The two write disjoint level ranges; the
  // main stream joins before L2L into levels hl..d.
  const int lmin = ctx->periodic ? 1 : 2;
  const int mlow = ctx->periodic ? 0 : 2;
  const int l2l_first = ctx->periodic ? 1 : 3;
  const int hl = std::max(lmin, d - 1);
  const T *Tm2m = static_cast<const T *>(ctx->m2m), *Tl2l = static_cast<const T *>(ctx->l2l);
  // M2M (up) into parent_level, or L2L (down) out of it.  The two deepest
  // levels' translations on the main stream run on the matrix cores; the
  // upper levels' ones on the second stream stay on the vector ALU, whose
  // blocks start in the main M2L launch's last round instead of taking
  // matrix-core cycles from it (measured: main M2L 0.94 -> 0.99 ms when the
  // upper levels used the matrix cores too).
  auto updown = [&](T *X, const T *Tab, int parent_level, bool up, hipStream_t s) {
    if constexpr (sizeof(T) == sizeof(float)) {
      const void *t16 = up ? ctx->m2m16 : ctx->l2l16;
      if (t16 && s == st) {
        launch_updown16(X, static_cast<const float *>(t16), parent_level, up, s);
        return;
      }
    }
    launch_updown<T>(X, Tab, p, KS, parent_level, up, s);
  };
  auto m2l = [&](int lo, int hi, hipStream_t s) {
    if (d < lmin || lo > hi) return;
    if constexpr (sizeof(T) == sizeof(float))
      launch_m2l_f32(Mc, Lc, static_cast<float *>(ctx->part), static_cast<const float *>(ctx->m2l), ctx->lists,
                     ctx->plan32, lo, hi, s);
    else
      launch_xlate_m2l<T>(Mc, Lc, static_cast<const T *>(ctx->m2l), ctx->lists, p, KS, d, ctx->periodic, lo, hi, s);
  };
  // only the deepest M2M (parent level d - 1) precedes the fork: the main M2L
  // needs multipoles of levels d - 1 and d only
  if (d - 1 >= mlow) updown(Mc, Tm2m, d - 1, true, st);
  ctx->mark(3);
  HIP_TRY(hipEventRecord(ctx->ev_fork, st), "fork");
  HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0), "fork");
  ctx->mark_side(0);
  if (ctx->periodic) launch_moments(ctx->qds, nleaf, ctx->qds + 5 * (int64_t)nleaf, ctx->side);
  for (int l = d - 2; l >= mlow; --l) updown(Mc, Tm2m, l, true, ctx->side);
  m2l(lmin, hl - 1, ctx->side);
  if (ctx->periodic) launch_lattice<T>(Mc, Lc, ctx->LamT, ncoef(p), ctx->qds + 5 * (int64_t)nleaf, ctx->geom, ctx->side);
  for (int l = l2l_first; l <= std::min(hl - 1, d); ++l) updown(Lc, Tl2l, l - 1, false, ctx->side);
  ctx->mark_side(1);
  HIP_TRY(hipEventRecord(ctx->ev_join, ctx->side), "join");
  ctx->mark(4);
  m2l(hl, d, st);
  ctx->mark(5);
  HIP_TRY(hipStreamWaitEvent(st, ctx->ev_join, 0), "join");
  for (int l = std::max(hl, l2l_first); l <= d; ++l) updown(Lc, Tl2l, l - 1, false, st);
  ctx->mark(6);
  launch_p2p<T>(tb.sorted, tb.sorted_lo, ctx->start, ctx->perm, Lc + level_offset(d) * KS, KS, ctx->geom, d, ctx->periodic, p, ctx->ke,
                static_cast<T *>(ctx->phi_sorted), F, pot, ctx->epart, st, ctx->p2p_mmax);
  ctx->mark(7);
  if (ctx->M > 0) {
    SiteArgs s = site_args<T>(ctx);
    const SiteIO<T> io{static_cast<const T *>(ctx->phi_sorted), nullptr, F, dvdl, ctx->dE_site, dedq, dvdl_qi,
                       ctx->site_ws, ctx->site_ws_stride};
    launch_site<T>(s, xyz, ctx->slot_of, ctx->geom, ctx->LamT, io, st);
  }
  ctx->mark(8);
  launch_finalize(ctx->epart, p2p_blocks<T>(d), ctx->dE_site, ctx->M, ctx->ke, E, E_qi, st);
  ctx->mark(9);
  if (ctx->prof_n < ctx->prof_max) ++ctx->prof_n;
  HIP_TRY(hipGetLastError(), "kernel launch");
  if (!dev) {
    if (a->energy) HIP_TRY(hipMemcpyAsync(a->energy, ctx->E, sizeof(double), hipMemcpyDeviceToHost, st), "copy energy");
    if (a->dvdl && ctx->M > 0)
      HIP_TRY(hipMemcpyAsync(a->dvdl, ctx->dvdl, sizeof(double) * ctx->nforms, hipMemcpyDeviceToHost, st), "copy dvdl");
    if (a->forces) HIP_TRY(hipMemcpyAsync(a->forces, ctx->F, sizeof(T) * 3 * N, hipMemcpyDeviceToHost, st), "copy forces");
    if (a->potential)
      HIP_TRY(hipMemcpyAsync(a->potential, ctx->pot, sizeof(T) * N, hipMemcpyDeviceToHost, st), "copy potential");
    if (dedq)
      HIP_TRY(hipMemcpyAsync(a->dedq, dedq, sizeof(double) * ctx->nfq, hipMemcpyDeviceToHost, st), "copy dE/dq");
    if (dvdl_qi)
      HIP_TRY(hipMemcpyAsync(a->dvdl_qi, dvdl_qi, sizeof(double) * ctx->nforms, hipMemcpyDeviceToHost, st),
              "copy dvdl_qi");
    if (E_qi) HIP_TRY(hipMemcpyAsync(a->energy_qi, E_qi, sizeof(double), hipMemcpyDeviceToHost, st), "copy energy");
    HIP_TRY(hipStreamSynchronize(st), "evaluation");
  }
  return MAHI_OK;
}

// Site correction on a potential from another solver: k_site reads ke * V from
// `potential` (user order) instead of the tree's potential; the energy is the
// sum of the per-site corrections.
// dE_site [M] and ws (M * site_ws_stride doubles, or null when the site pass
// keeps its work arrays in local memory) are the call's scratch.
template <class T>
mahi_status correct_impl(mahi_ctx *ctx, const mahi_correct_args *a, double *dE_site, double *ws) {
  const bool dev = (a->flags & MAHI_DEVICE_IO) != 0;
  const int64_t N = ctx->N;
  hipStream_t st = ctx->stream;
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  const T *xyz = static_cast<const T *>(a->xyz), *pot = static_cast<const T *>(a->potential);
  T *F = static_cast<T *>(a->forces);
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(ctx->xyz, a->xyz, sizeof(T) * 3 * N, hipMemcpyHostToDevice, st), "copy positions");
    HIP_TRY(hipMemcpyAsync(ctx->pot, a->potential, sizeof(T) * N, hipMemcpyHostToDevice, st), "copy potential");
    xyz = static_cast<const T *>(ctx->xyz);
    pot = static_cast<const T *>(ctx->pot);
    if (F) {
      HIP_TRY(hipMemcpyAsync(ctx->F, a->forces, sizeof(T) * 3 * N, hipMemcpyHostToDevice, st), "copy forces");
      F = static_cast<T *>(ctx->F);
    }
  }
  double *E = (dev && a->energy) ? a->energy : ctx->E;
  double *dvdl = a->dvdl ? (dev ? a->dvdl : ctx->dvdl) : nullptr;
  double *dedq = a->dedq ? (dev ? a->dedq : ctx->dedq) : nullptr;
  if (ctx->M > 0) {
    SiteArgs s = site_args<T>(ctx);
    const SiteIO<T> io{nullptr, pot, F, dvdl, dE_site, dedq, nullptr, ws, ctx->site_ws_stride};
    launch_site<T>(s, xyz, ctx->slot_of, ctx->geom, ctx->LamT, io, st);
  }
  launch_finalize(nullptr, 0, dE_site, ctx->M, ctx->ke, E, nullptr, st);
  HIP_TRY(hipGetLastError(), "kernel launch");
  if (!dev) {
    if (a->energy) HIP_TRY(hipMemcpyAsync(a->energy, ctx->E, sizeof(double), hipMemcpyDeviceToHost, st), "copy energy");
    if (dvdl)
      HIP_TRY(hipMemcpyAsync(a->dvdl, dvdl, sizeof(double) * ctx->nforms, hipMemcpyDeviceToHost, st), "copy dvdl");
    if (dedq) HIP_TRY(hipMemcpyAsync(a->dedq, dedq, sizeof(double) * ctx->nfq, hipMemcpyDeviceToHost, st), "copy dE/dq");
    if (F) HIP_TRY(hipMemcpyAsync(a->forces, F, sizeof(T) * 3 * N, hipMemcpyDeviceToHost, st), "copy forces");
    HIP_TRY(hipStreamSynchronize(st), "correction");
  }
  return MAHI_OK;
}

template <class T>
bool all_finite(const void *p, int64_t n) {
  const T *x = static_cast<const T *>(p);
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

#define BATCH_TRY(expr, what)                                                                \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) return b->fail(MAHI_EDEVICE, std::string(what) + ": " + hip_msg(_e)); \
  } while (0)

void batch_drop_graph(mahi_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->captured.clear();
}

bool same_args(const mahi_eval_args &a, const mahi_eval_args &c) {
  return a.xyz == c.xyz && a.energy == c.energy && a.forces == c.forces && a.dvdl == c.dvdl &&
         a.potential == c.potential && a.flags == c.flags && a.dedq == c.dedq && a.energy_qi == c.energy_qi &&
         a.dvdl_qi == c.dvdl_qi;
}

// Whether a batch can run packed: float32, periodic, one order (shared
// tables), and sites whose work arrays fit in local memory at the batch's
// largest site.
bool packed_ok(const std::vector<mahi_ctx *> &c, int &maxa, int &maxf) {
  maxa = 1;
  maxf = 1;
  for (const mahi_ctx *x : c) {
    if (x->prec != 32 || !x->periodic || x->p != c[0]->p || x->d > 7) return false;
    maxa = std::max(maxa, x->maxa);
    maxf = std::max(maxf, x->maxf);
  }
  return site_in_lds(c[0]->p, maxa, maxf);
}

#define PACK_TRY(expr, what)                                                             \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) return std::string(what) + ": " + hip_msg(_e);                 \
  } while (0)

// Allocate the packed batch's buffers and block ranges and fill the
// descriptor template (offsets, tables, plans); "" on success.
std::string packed_setup(mahi_batch *b, int maxa, int maxf) {
  const auto &c = b->ctxs;
  const int ns = (int)c.size(), p = c[0]->p, K = ncoef(p), KS = c[0]->KS;
  PackedPlan &pp = b->pp;
  pp.nsys = ns;
  pp.p = p;
  pp.K = K;
  pp.KS = KS;
  int64_t atoms = 0, boxes = 0;
  int leaves = 0, tiles = 0;
  b->sys_host.assign(ns, PackedSys{});
  for (int i = 0; i < ns; ++i) {
    PackedSys &S = b->sys_host[i];
    const mahi_ctx *x = c[i];
    S.atom_off = atoms;
    S.n_atoms = x->N;
    S.box_off = boxes;
    S.leaf_off = leaves;
    S.d = x->d;
    S.nleaf = 1 << (3 * x->d);
    S.n_sites = x->M;
    S.ke = x->ke;
    atoms += x->N;
    boxes += level_offset(x->d + 1);
    leaves += S.nleaf;
    tiles += x->plan32.ntiles;
    pp.dmax = std::max(pp.dmax, x->d);
  }
  if (atoms > (int64_t)0x7fffffff - 1) return "the batch holds more than 2^31 - 2 atoms";
  pp.n_atoms = atoms;
  pp.nleaf = leaves;
  pp.nbox = boxes + 1;  // + the all-zero row
  // operator ranges: the fluid makespan model of the single-system plan on the batch's tiles
  const M2LPlan &p0 = c[0]->plan32;
  {
    const double slots = 2.0 * (c[0]->n_cu > 0 ? c[0]->n_cu : 256);
    const double steps = (double)kListLen * p0.nkc, work = (double)tiles * p0.ngroups * steps;
    double best = 1e300;
    pp.nsplit = 1;
    for (int sp = 1; sp <= kM2LMaxSplit; ++sp) {
      const double item = steps / sp;
      const double cost = std::max(work / slots + 0.5 * item, item) + steps / 32.0 * sp;
      if (cost < best - 1e-9) {
        best = cost;
        pp.nsplit = sp;
      }
    }
  }
  int chunk = (int)(16384 / (K * sizeof(float)));
  pp.chunk = std::max(1, std::min(chunk, 32));
  const int np_up = updown_np<float>(KS, true), np_dn = updown_np<float>(KS, false);
  // block ranges of every per-system stage
  std::vector<std::vector<int>> firsts;
  auto stage = [&](PackedStage &stg, auto blocks_of) {
    std::vector<int> f(ns + 1, 0);
    for (int i = 0; i < ns; ++i) f[i + 1] = f[i] + blocks_of(i);
    stg.blocks = f[ns];
    firsts.push_back(std::move(f));
  };
  std::vector<PackedStage *> stages;
  stage(pp.atoms, [&](int i) { return (int)((c[i]->N + 255) / 256); });
  stages.push_back(&pp.atoms);
  stage(pp.leaves, [&](int i) { return b->sys_host[i].nleaf; });
  stages.push_back(&pp.leaves);
  stage(pp.m2l, [&](int i) { return c[i]->plan32.ntiles * pp.nsplit * p0.ngroups; });
  stages.push_back(&pp.m2l);
  stage(pp.sites, [&](int i) { return c[i]->M; });
  stages.push_back(&pp.sites);
  for (int j = 1; j <= pp.dmax; ++j) {
    stage(pp.up[j - 1], [&](int i) {
      const int pl = c[i]->d - j;
      return pl < 0 ? 0 : (int)(((int64_t(1) << (3 * pl)) + np_up - 1) / np_up);
    });
    stages.push_back(&pp.up[j - 1]);
    stage(pp.down[j - 1], [&](int i) {
      return j > c[i]->d ? 0 : (int)(((int64_t(1) << (3 * (j - 1))) + np_dn - 1) / np_dn);
    });
    stages.push_back(&pp.down[j - 1]);
  }
  int *firsts_dev = nullptr;
  PACK_TRY(b->alloc(firsts_dev, sizeof(int) * (ns + 1) * firsts.size()), "alloc block ranges");
  for (size_t k = 0; k < firsts.size(); ++k) {
    PACK_TRY(hipMemcpy(firsts_dev + k * (ns + 1), firsts[k].data(), sizeof(int) * (ns + 1), hipMemcpyHostToDevice),
             "upload block ranges");
    stages[k]->first = firsts_dev + k * (ns + 1);
  }
  // buffers
  const size_t N = (size_t)atoms, L = (size_t)leaves, B = (size_t)pp.nbox;
  PACK_TRY(b->alloc(pp.key, sizeof(int) * N), "alloc keys");
  PACK_TRY(b->alloc(pp.rank, sizeof(int) * N), "alloc ranks");
  PACK_TRY(b->alloc(pp.tmp, sizeof(int) * N), "alloc scatter");
  PACK_TRY(b->alloc(pp.perm, sizeof(int) * N), "alloc perm");
  PACK_TRY(b->alloc(pp.slot_of, sizeof(int) * N), "alloc slot map");
  PACK_TRY(b->alloc(pp.count, sizeof(int) * L), "alloc counts");
  PACK_TRY(hipMemset(pp.count, 0, sizeof(int) * L), "zero counts");  // k_scan clears them after each use
  PACK_TRY(b->alloc(pp.start, sizeof(int) * (L + 1)), "alloc starts");
  PACK_TRY(b->alloc(pp.packed, sizeof(Atom4<float>) * N), "alloc packed atoms");
  PACK_TRY(b->alloc(pp.sorted, sizeof(Atom4<float>) * N), "alloc sorted atoms");
  PACK_TRY(b->alloc(pp.phi_sorted, sizeof(float) * N), "alloc potentials");
  PACK_TRY(b->alloc(pp.Mc, sizeof(float) * B * KS), "alloc multipoles");
  PACK_TRY(b->alloc(pp.Lc, sizeof(float) * B * KS), "alloc locals");
  PACK_TRY(b->alloc(pp.part, sizeof(float) * pp.nsplit * B * KS), "alloc M2L partials");
  // pads, level-0 partials and the zero row stay zero (never written)
  PACK_TRY(hipMemset(pp.Mc, 0, sizeof(float) * B * KS), "zero multipoles");
  PACK_TRY(hipMemset(pp.Lc, 0, sizeof(float) * B * KS), "zero locals");
  PACK_TRY(hipMemset(pp.part, 0, sizeof(float) * pp.nsplit * B * KS), "zero partials");
  PACK_TRY(b->alloc(pp.qds, sizeof(double) * 5 * L), "alloc moments");
  PACK_TRY(b->alloc(pp.epart, sizeof(double) * L), "alloc energy partials");
  PACK_TRY(b->alloc(b->sys_dev, sizeof(PackedSys) * ns), "alloc descriptors");
  pp.sys = b->sys_dev;
  // tables of the first context (one order: the same tables for every system)
  pp.m2l_tab = static_cast<const float *>(c[0]->m2l);
  pp.m2m = static_cast<const float *>(c[0]->m2m);
  pp.l2l = static_cast<const float *>(c[0]->l2l);
  pp.lists = c[0]->lists;
  pp.LamT = c[0]->LamT;
  const int site_dloc = site_lds_bytes(p, maxa, maxf, true) + kSiteStaticLds <= 65536 ? 1 : 0;
  pp.site_lds = site_lds_bytes(p, maxa, maxf, site_dloc != 0);
  for (int i = 0; i < ns; ++i) {
    PackedSys &S = b->sys_host[i];
    mahi_ctx *x = c[i];
    S.qt = static_cast<const float *>(x->qt);
    S.geom = x->geom;
    S.site = site_args<float>(x);
    S.site.maxa = maxa;
    S.site.maxf = maxf;
    S.site.dloc = site_dloc;
    S.plan = x->plan32;
    S.plan.tile0 = 0;
    S.plan.tile_run = x->plan32.ntiles;
    S.plan.nsplit = pp.nsplit;
    S.plan.nbox = pp.nbox;                 // stride of the partial arrays
    S.plan.zbox = boxes - S.box_off;       // the batch's zero row, relative to the system
    S.p2p.d = x->d;
    S.p2p.periodic = 1;
    S.p2p.p = p;
    S.p2p.K = K;
    S.p2p.KS = KS;
    S.p2p.mmax = 3;
    S.p2p.dloc = (size_t)4 * K * sizeof(float) <= 16384 ? 1 : 0;
    S.p2p.ke = x->ke;
  }
  return "";
}

// Point the device descriptors at this call's arguments (waits for the
// batch's stream first: a previous launch may still read them).
mahi_status packed_table(mahi_batch *b, const mahi_eval_args *args) {
  const size_t ns = b->ctxs.size();
  bool same = b->table.size() == ns;
  for (size_t i = 0; same && i < ns; ++i) same = same_args(args[i], b->table[i]);
  if (same) return MAHI_OK;
  for (size_t i = 0; i < ns; ++i) {
    PackedSys &S = b->sys_host[i];
    mahi_ctx *x = b->ctxs[i];
    const mahi_eval_args &a = args[i];
    S.xyz = static_cast<const float *>(a.xyz);
    S.F = static_cast<float *>(a.forces);
    S.pot = static_cast<float *>(a.potential);
    S.E = a.energy ? a.energy : x->E;
    S.E_qi = a.energy_qi;
    S.io = SiteIO<float>{b->pp.phi_sorted, nullptr, S.F, (x->M > 0 && a.dvdl) ? a.dvdl : x->dvdl, x->dE_site,
                         x->M > 0 ? a.dedq : nullptr, x->M > 0 ? a.dvdl_qi : nullptr, nullptr, 0};
  }
  BATCH_TRY(hipStreamSynchronize(b->root), "batch stream");
  BATCH_TRY(hipMemcpy(b->sys_dev, b->sys_host.data(), sizeof(PackedSys) * ns, hipMemcpyHostToDevice),
            "upload descriptors");
  b->table.assign(args, args + ns);
  batch_drop_graph(b);
  return MAHI_OK;
}

// Fork from the origin stream into every context's stream, evaluate, join back.
mahi_status batch_issue(mahi_batch *b, const mahi_eval_args *args) {
  BATCH_TRY(hipEventRecord(b->fork, b->root), "batch fork");
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    mahi_ctx *ctx = b->ctxs[i];
    BATCH_TRY(hipStreamWaitEvent(ctx->stream, b->fork, 0), "batch fork");
    const mahi_status st = ctx->prec == 32 ? eval_impl<float>(ctx, &args[i]) : eval_impl<double>(ctx, &args[i]);
    if (st != MAHI_OK) return b->fail(st, "system " + std::to_string(i) + ": " + ctx->err);
    BATCH_TRY(hipEventRecord(b->joins[i], ctx->stream), "batch join");
    BATCH_TRY(hipStreamWaitEvent(b->root, b->joins[i], 0), "batch join");
  }
  return MAHI_OK;
}

void free_ctx(mahi_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->side) (void)hipStreamSynchronize(ctx->side);
  for (auto &e : ctx->prof_events) (void)hipEventDestroy(e);
  for (auto &b : ctx->bufs) (void)hipFree(b.p);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

}  // namespace

extern "C" {

const char *mahi_strerror(mahi_status s) {
  switch (s) {
    case MAHI_OK: return "ok";
    case MAHI_EINVAL: return "invalid argument";
    case MAHI_ENOMEM: return "out of memory";
    case MAHI_EDEVICE: return "device error";
    case MAHI_ERANGE: return "value out of supported range";
    case MAHI_ESTATE: return "call out of order";
    case MAHI_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char *mahi_last_error(const mahi_ctx *ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->err.c_str();
}

mahi_status mahi_create(mahi_ctx **out, const mahi_box *box, int64_t n_atoms, const double *charges,
                        const mahi_sites *sites, const mahi_opts *opts) {
  g_create_error.clear();
  auto bad = [](mahi_status s, const std::string &m) {
    g_create_error = m;
    return s;
  };
  if (!out) return bad(MAHI_EINVAL, "out is NULL");
  *out = nullptr;
  if (!box || !opts || !charges) return bad(MAHI_EINVAL, "box, opts and charges must not be NULL");
  if (n_atoms < 1 || n_atoms > (int64_t)0x7fffffff - 1) return bad(MAHI_ERANGE, "n_atoms must be in 1..2^31-2");
  if (box->periodic != 0 && box->periodic != 1) return bad(MAHI_EINVAL, "box.periodic must be 0 or 1");
  if (box->periodic && !(is_fin(box->edge) && box->edge > 0)) return bad(MAHI_EINVAL, "periodic box edge must be > 0");
  if (opts->order < 1 || opts->order > kMaxOrder) return bad(MAHI_ERANGE, "order must be in 1..20");
  if (opts->depth < 0 || opts->depth > 7) return bad(MAHI_ERANGE, "depth must be in 0..7");
  if (opts->precision != 32 && opts->precision != 64) return bad(MAHI_EINVAL, "precision must be 32 or 64");
  if (!is_fin(opts->coulomb_k)) return bad(MAHI_EINVAL, "coulomb_k must be finite");
  for (int64_t i = 0; i < n_atoms; ++i)
    if (!is_fin(charges[i])) return bad(MAHI_EINVAL, "non-finite charge");
  std::vector<double> q_env(charges, charges + n_atoms);
  std::vector<int> atom_off{0}, form_off{0}, fq_off, site_atoms;
  std::vector<double> fq;
  int maxa = 0, maxf = 0;
  const int M = sites ? sites->n_sites : 0;
  if (sites) {
    if (M < 0) return bad(MAHI_EINVAL, "n_sites must be >= 0");
    if (M > 0 && (!sites->forms_per_site || !sites->atoms_per_site || !sites->site_atoms || !sites->form_charges))
      return bad(MAHI_EINVAL, "site arrays must not be NULL");
    std::vector<char> used(n_atoms, 0);
    int64_t fo = 0;
    for (int s = 0; s < M; ++s) {
      const int nf = sites->forms_per_site[s], na = sites->atoms_per_site[s];
      if (nf < 1 || nf > kMaxSiteForms) return bad(MAHI_ERANGE, "forms per site must be in 1..16");
      if (na < 1 || na > kMaxSiteAtoms) return bad(MAHI_ERANGE, "atoms per site must be in 1..32");
      maxa = std::max(maxa, na);
      maxf = std::max(maxf, nf);
      for (int i = 0; i < na; ++i) {
        const int at = sites->site_atoms[atom_off.back() + i];
        if (at < 0 || at >= n_atoms) return bad(MAHI_EINVAL, "site atom index out of range");
        if (used[at]) return bad(MAHI_EINVAL, "site atoms overlap");
        used[at] = 1;
        site_atoms.push_back(at);
      }
      fq_off.push_back((int)fo);
      for (int k = 0; k < nf * na; ++k) {
        const double v = sites->form_charges[fo + k];
        if (!is_fin(v)) return bad(MAHI_EINVAL, "non-finite form charge");
        fq.push_back(v);
      }
      fo += (int64_t)nf * na;
      atom_off.push_back(atom_off.back() + na);
      form_off.push_back(form_off.back() + nf);
    }
    for (size_t i = 0; i < site_atoms.size(); ++i) q_env[site_atoms[i]] = 0.0;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return bad(MAHI_EDEVICE, "no HIP device");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return bad(MAHI_EDEVICE, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return bad(MAHI_EDEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return bad(MAHI_EDEVICE, std::string("built for gfx950, found ") + prop.gcnArchName);
  {
    // the allocation-free correction's static scratch: its address on this
    // device, looked up once with the device current
    void *sp = nullptr;
    const hipError_t e = static_scratch(dev, &sp);
    if (e != hipSuccess) return bad(MAHI_EDEVICE, std::string("static scratch: ") + hip_msg(e));
  }
  mahi_ctx *ctx = new (std::nothrow) mahi_ctx;
  if (!ctx) return bad(MAHI_ENOMEM, "host allocation failed");
  ctx->N = n_atoms;
  ctx->periodic = box->periodic;
  ctx->edge = box->edge;
  ctx->p = opts->order;
  ctx->d = opts->depth;
  ctx->prec = opts->precision;
  ctx->ke = opts->coulomb_k > 0 ? opts->coulomb_k : kDefaultKe;
  ctx->device = dev;
  ctx->n_cu = prop.multiProcessorCount;
  ctx->M = M;
  ctx->nforms = form_off.back();
  ctx->nsite_atoms = (int)site_atoms.size();
  ctx->nfq = (int64_t)fq.size();
  ctx->maxa = maxa;
  ctx->maxf = maxf;
  ctx->lambda_set = (M == 0);
  if (opts->hip_stream) {
    ctx->stream = static_cast<hipStream_t>(opts->hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return bad(MAHI_EDEVICE, "stream creation failed");
    }
    ctx->own_stream = true;
  }
  mahi_status s = ctx->prec == 32 ? setup_device<float>(ctx, q_env, atom_off, form_off, fq_off, site_atoms, fq)
                                   : setup_device<double>(ctx, q_env, atom_off, form_off, fq_off, site_atoms, fq);
  if (s != MAHI_OK) {
    g_create_error = ctx->err;
    free_ctx(ctx);
    return s;
  }
  *out = ctx;
  return MAHI_OK;
}

mahi_status mahi_set_lambda(mahi_ctx *ctx, const double *lt) {
  if (!ctx) return MAHI_EINVAL;
  if (ctx->M == 0) {
    ctx->lambda_set = true;
    return MAHI_OK;
  }
  if (!lt) return ctx->fail(MAHI_EINVAL, "lambda_tilde is NULL");
  for (int i = 0; i < ctx->nforms; ++i)
    if (!is_fin(lt[i])) return ctx->fail(MAHI_EINVAL, "non-finite lambda_tilde");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  HIP_TRY(hipMemcpyAsync(ctx->lam, lt, sizeof(double) * ctx->nforms, hipMemcpyHostToDevice, ctx->stream), "copy lambda");
  if (ctx->prec == 32) {
    SiteArgs s = site_args<float>(ctx);
    launch_charge_scale<float>(s, ctx->lam, static_cast<float *>(ctx->qt), ctx->stream);
  } else {
    SiteArgs s = site_args<double>(ctx);
    launch_charge_scale<double>(s, ctx->lam, static_cast<double *>(ctx->qt), ctx->stream);
  }
  HIP_TRY(hipGetLastError(), "charge scaling launch");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "charge scaling");
  ctx->lambda_set = true;
  return MAHI_OK;
}

mahi_status mahi_eval(mahi_ctx *ctx, const mahi_eval_args *a) {
  if (!ctx) return MAHI_EINVAL;
  if (!a || !a->xyz) return ctx->fail(MAHI_EINVAL, "args and args->xyz must not be NULL");
  if (a->flags & ~MAHI_DEVICE_IO) return ctx->fail(MAHI_EINVAL, "unknown flags");
  if (!ctx->lambda_set) return ctx->fail(MAHI_ESTATE, "mahi_set_lambda must be called before mahi_eval");
  if (!(a->flags & MAHI_DEVICE_IO)) {
    const bool ok = ctx->prec == 32 ? all_finite<float>(a->xyz, 3 * ctx->N) : all_finite<double>(a->xyz, 3 * ctx->N);
    if (!ok) return ctx->fail(MAHI_EINVAL, "non-finite coordinate");
  }
  return ctx->prec == 32 ? eval_impl<float>(ctx, a) : eval_impl<double>(ctx, a);
}

mahi_status mahi_correct(mahi_ctx *ctx, const mahi_correct_args *a) {
  if (!ctx) return MAHI_EINVAL;
  if (!a || !a->xyz || !a->potential) return ctx->fail(MAHI_EINVAL, "args, args->xyz and args->potential must not be NULL");
  if (a->flags & ~MAHI_DEVICE_IO) return ctx->fail(MAHI_EINVAL, "unknown flags");
  if (!ctx->lambda_set) return ctx->fail(MAHI_ESTATE, "mahi_set_lambda must be called before mahi_correct");
  if (!(a->flags & MAHI_DEVICE_IO)) {
    const bool f32 = ctx->prec == 32;
    if (!(f32 ? all_finite<float>(a->xyz, 3 * ctx->N) : all_finite<double>(a->xyz, 3 * ctx->N)))
      return ctx->fail(MAHI_EINVAL, "non-finite coordinate");
    if (!(f32 ? all_finite<float>(a->potential, ctx->N) : all_finite<double>(a->potential, ctx->N)))
      return ctx->fail(MAHI_EINVAL, "non-finite potential");
  }
  return ctx->prec == 32 ? correct_impl<float>(ctx, a, ctx->dE_site, ctx->site_ws)
                         : correct_impl<double>(ctx, a, ctx->dE_site, ctx->site_ws);
}

mahi_status mahi_correct_noalloc(mahi_ctx *ctx, const mahi_correct_args *a) {
  if (!ctx) return MAHI_EINVAL;
  if (!a || !a->xyz || !a->potential) return ctx->fail(MAHI_EINVAL, "args, args->xyz and args->potential must not be NULL");
  if (a->flags != MAHI_DEVICE_IO)
    return ctx->fail(MAHI_EINVAL, "mahi_correct_noalloc takes device pointers only (flags = MAHI_DEVICE_IO)");
  if (!ctx->lambda_set) return ctx->fail(MAHI_ESTATE, "mahi_set_lambda must be called before mahi_correct_noalloc");
  // scratch: per-site energies (rounded up to 256 bytes), then the site pass's
  // work arrays when they exceed local memory
  const size_t de_bytes = (sizeof(double) * (size_t)ctx->M + 255) / 256 * 256;
  const size_t ws_bytes = ctx->site_ws ? sizeof(double) * (size_t)ctx->site_ws_stride * ctx->M : 0;
  if (de_bytes + ws_bytes > kStaticScratchBytes)
    return ctx->fail(MAHI_ERANGE, "the correction needs " + std::to_string(de_bytes + ws_bytes) +
                                      " bytes of scratch; the static scratch holds " +
                                      std::to_string(kStaticScratchBytes));
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  void *sp = nullptr;
  HIP_TRY(static_scratch(ctx->device, &sp), "static scratch");
  double *dE_site = static_cast<double *>(sp);
  double *ws = ws_bytes ? reinterpret_cast<double *>(static_cast<unsigned char *>(sp) + de_bytes) : nullptr;
  return ctx->prec == 32 ? correct_impl<float>(ctx, a, dE_site, ws) : correct_impl<double>(ctx, a, dE_site, ws);
}

mahi_status mahi_set_form_charges(mahi_ctx *ctx, const double *form_charges) {
  if (!ctx) return MAHI_EINVAL;
  if (ctx->M == 0) return MAHI_OK;
  if (!form_charges) return ctx->fail(MAHI_EINVAL, "form_charges is NULL");
  if (!all_finite<double>(form_charges, ctx->nfq)) return ctx->fail(MAHI_EINVAL, "non-finite form charge");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  HIP_TRY(hipMemcpyAsync(ctx->fq, form_charges, sizeof(double) * ctx->nfq, hipMemcpyHostToDevice, ctx->stream),
          "copy form charges");
  if (ctx->lambda_set) {
    if (ctx->prec == 32)
      launch_charge_scale<float>(site_args<float>(ctx), ctx->lam, static_cast<float *>(ctx->qt), ctx->stream);
    else
      launch_charge_scale<double>(site_args<double>(ctx), ctx->lam, static_cast<double *>(ctx->qt), ctx->stream);
    HIP_TRY(hipGetLastError(), "charge scaling launch");
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream), "form charges");
  return MAHI_OK;
}

mahi_status mahi_lambda_tilde(int n_lambda, const double *lambda, double *lt) {
  if (n_lambda < 1 || n_lambda > 4) return MAHI_ERANGE;
  if (!lambda || !lt) return MAHI_EINVAL;
  for (int k = 0; k < n_lambda; ++k)
    if (!is_fin(lambda[k])) return MAHI_EINVAL;
  // lt over forms 0..2^k-1 doubles at each k: forms with bit k clear take
  // (1 - lambda_k), the others lambda_k
  lt[0] = 1.0;
  for (int k = 0; k < n_lambda; ++k) {
    const int h = 1 << k;
    for (int r = 0; r < h; ++r) {
      lt[h + r] = lt[r] * lambda[k];
      lt[r] *= 1.0 - lambda[k];
    }
  }
  return MAHI_OK;
}

mahi_status mahi_dlambda(int n_lambda, const double *lambda, const double *dvdl, double *dlambda) {
  if (n_lambda < 1 || n_lambda > 4) return MAHI_ERANGE;
  if (!lambda || !dvdl || !dlambda) return MAHI_EINVAL;
  const int nf = 1 << n_lambda;
  for (int k = 0; k < n_lambda; ++k)
    if (!is_fin(lambda[k])) return MAHI_EINVAL;
  for (int r = 0; r < nf; ++r)
    if (!is_fin(dvdl[r])) return MAHI_EINVAL;
  for (int k = 0; k < n_lambda; ++k) {
    // d lt_r / d lambda_k = +-(product of the other factors): the weights of
    // the remaining n_lambda - 1 lambdas, indexed by r with bit k removed
    double other[8];
    int n_other = 0;
    for (int j = 0; j < n_lambda; ++j)
      if (j != k) other[n_other++] = lambda[j];
    double w[8];
    w[0] = 1.0;
    for (int j = 0; j < n_other; ++j) {
      const int h = 1 << j;
      for (int r = 0; r < h; ++r) {
        w[h + r] = w[r] * other[j];
        w[r] *= 1.0 - other[j];
      }
    }
    double acc = 0.0;
    for (int r = 0; r < nf; ++r) {
      const int lo = r & ((1 << k) - 1), hi = r >> (k + 1);
      const double f = w[lo | (hi << k)];
      acc += ((r >> k) & 1) ? f * dvdl[r] : -f * dvdl[r];
    }
    dlambda[k] = acc;
  }
  return MAHI_OK;
}

void mahi_destroy(mahi_ctx *ctx) { free_ctx(ctx); }

mahi_status mahi_get_stream(const mahi_ctx *ctx, void **stream) {
  if (!ctx || !stream) return MAHI_EINVAL;
  *stream = static_cast<void *>(ctx->stream);
  return MAHI_OK;
}

mahi_status mahi_info(const mahi_ctx *ctx, int64_t *n_atoms, int32_t *n_sites, int32_t *n_forms, int *order, int *depth,
                      int *precision) {
  if (!ctx) return MAHI_EINVAL;
  if (n_atoms) *n_atoms = ctx->N;
  if (n_sites) *n_sites = ctx->M;
  if (n_forms) *n_forms = ctx->nforms;
  if (order) *order = ctx->p;
  if (depth) *depth = ctx->d;
  if (precision) *precision = ctx->prec;
  return MAHI_OK;
}

const char *mahi_stage_name(int stage) {
  static const char *names[MAHI_N_STAGES] = {"tree", "p2m", "m2m", "upper_levels", "m2l", "l2l", "p2p_l2p", "site", "energy"};
  return (stage >= 0 && stage < MAHI_N_STAGES) ? names[stage] : "unknown";
}

mahi_status mahi_profile_begin(mahi_ctx *ctx, int max_evals) {
  if (!ctx) return MAHI_EINVAL;
  if (max_evals < 1 || max_evals > 100000) return ctx->fail(MAHI_ERANGE, "max_evals must be in 1..100000");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "synchronise");
  for (auto &e : ctx->prof_events) (void)hipEventDestroy(e);
  ctx->prof_events.assign((size_t)max_evals * mahi_ctx::kSlots, nullptr);
  for (auto &e : ctx->prof_events) HIP_TRY(hipEventCreate(&e), "event create");
  ctx->prof_max = max_evals;
  ctx->prof_n = 0;
  return MAHI_OK;
}

mahi_status mahi_profile_end(mahi_ctx *ctx, double *stage_ms, int *n_evals) {
  if (!ctx || !stage_ms) return MAHI_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "synchronise");
  for (int s = 0; s < MAHI_N_STAGES; ++s) stage_ms[s] = 0.0;
  HIP_TRY(hipStreamSynchronize(ctx->side), "synchronise");
  for (int e = 0; e < ctx->prof_n; ++e)
    for (int s = 0; s < MAHI_N_STAGES; ++s) {
      // stage s between main-stream boundaries s and s + 1, except stage 3 (the
      // upper levels), which runs on the side stream between its own two events
      const size_t base = (size_t)e * mahi_ctx::kSlots;
      const bool side = s == 3;
      const size_t a0 = side ? base + MAHI_N_STAGES + 1 : base + s;
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ctx->prof_events[a0], ctx->prof_events[a0 + 1]), "event timing");
      stage_ms[s] += ms;
    }
  ctx->prof_totals.assign(ctx->prof_n, 0.0);
  for (int e = 0; e < ctx->prof_n; ++e) {
    const size_t base = (size_t)e * mahi_ctx::kSlots;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->prof_events[base], ctx->prof_events[base + MAHI_N_STAGES]), "event timing");
    ctx->prof_totals[e] = ms;
  }
  ctx->prof_done = true;
  if (ctx->prof_n > 0)
    for (int s = 0; s < MAHI_N_STAGES; ++s) stage_ms[s] /= ctx->prof_n;
  if (n_evals) *n_evals = ctx->prof_n;
  for (auto &e : ctx->prof_events) (void)hipEventDestroy(e);
  ctx->prof_events.clear();
  ctx->prof_max = ctx->prof_n = 0;
  return MAHI_OK;
}

mahi_status mahi_profile_eval_times(const mahi_ctx *ctx, double *eval_ms, int max, int *n) {
  if (!ctx || !n || max < 0 || (max > 0 && !eval_ms)) return MAHI_EINVAL;
  if (!ctx->prof_done) return MAHI_ESTATE;
  const int m = std::min<int>(max, (int)ctx->prof_totals.size());
  for (int i = 0; i < m; ++i) eval_ms[i] = ctx->prof_totals[i];
  *n = m;
  return MAHI_OK;
}

mahi_status mahi_debug_copy(mahi_ctx *ctx, int which, void *host_out, int64_t count) {
  if (!ctx || !host_out || count < 0) return MAHI_EINVAL;
  const size_t el = ctx->prec == 32 ? sizeof(float) : sizeof(double);
  const int K = ncoef(ctx->p), KS = ctx->KS;
  const int64_t nbox = level_offset(ctx->d + 1);
  const void *src = nullptr;
  size_t bytes = 0;
  switch (which) {
    case 0: src = ctx->Mc; bytes = el * nbox * K; break;
    case 1: src = ctx->Lc; bytes = el * nbox * K; break;
    case 2: src = ctx->start; bytes = sizeof(int) * ((size_t(1) << (3 * ctx->d)) + 1); break;
    case 3: src = ctx->perm; bytes = sizeof(int) * ctx->N; break;
    case 4: src = ctx->sorted; bytes = 4 * el * ctx->N; break;
    default: return ctx->fail(MAHI_EINVAL, "unknown buffer");
  }
  const size_t want = (which == 2 || which == 3 ? sizeof(int) : el) * (size_t)count;
  if (want > bytes) return ctx->fail(MAHI_ERANGE, "count exceeds the buffer");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "synchronise");
  if ((which == 0 || which == 1) && KS != K) {
    // boxes are stored with stride KS: copy whole rows, then drop the padding
    const int64_t nb = (count + K - 1) / K;
    std::vector<unsigned char> rows((size_t)nb * KS * el);
    HIP_TRY(hipMemcpy(rows.data(), src, rows.size(), hipMemcpyDeviceToHost), "copy");
    unsigned char *out = static_cast<unsigned char *>(host_out);
    for (int64_t i = 0; i < count; ++i) {
      const int64_t b = i / K, k = i - b * K;
      std::memcpy(out + (size_t)i * el, rows.data() + ((size_t)b * KS + k) * el, el);
    }
    return MAHI_OK;
  }
  HIP_TRY(hipMemcpy(host_out, src, want, hipMemcpyDeviceToHost), "copy");
  return MAHI_OK;
}

mahi_status mahi_batch_create(mahi_batch **out, mahi_ctx *const *ctxs, int n_ctx, int flags, void *hip_stream) {
  g_create_error.clear();
  if (!out) return MAHI_EINVAL;
  *out = nullptr;
  if (!ctxs || n_ctx < 1) {
    g_create_error = "ctxs must hold at least one context";
    return MAHI_EINVAL;
  }
  if (flags & ~(int)(MAHI_BATCH_GRAPH | MAHI_BATCH_PACKED)) {
    g_create_error = "unknown batch flags";
    return MAHI_EINVAL;
  }
  const bool want_graph = (flags & MAHI_BATCH_GRAPH) != 0, want_packed = (flags & MAHI_BATCH_PACKED) != 0;
  for (int i = 0; i < n_ctx; ++i) {
    if (!ctxs[i]) {
      g_create_error = "NULL context";
      return MAHI_EINVAL;
    }
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) {
        g_create_error = "a context appears twice";
        return MAHI_EINVAL;
      }
    if (ctxs[i]->device != ctxs[0]->device) {
      g_create_error = "contexts on different devices";
      return MAHI_EINVAL;
    }
  }
  if (want_graph && !want_packed) {
    // The fork/join of separate contexts is not captured: its first capture
    // and launch ended in a host segmentation fault whose cause is not shown.
    g_create_error = "graph capture needs a packed batch (MAHI_BATCH_PACKED)";
    return MAHI_EUNSUPPORTED;
  }
  int maxa = 1, maxf = 1;
  if (want_packed && !packed_ok(std::vector<mahi_ctx *>(ctxs, ctxs + n_ctx), maxa, maxf)) {
    g_create_error = "a packed batch needs float32 periodic contexts of one order (at most 8) whose sites fit in "
                     "local memory";
    return MAHI_EUNSUPPORTED;
  }
  mahi_batch *b = new (std::nothrow) mahi_batch;
  if (!b) return MAHI_ENOMEM;
  b->ctxs.assign(ctxs, ctxs + n_ctx);
  b->device = ctxs[0]->device;
  b->use_graph = want_graph;
  b->packed = want_packed;
  auto bad = [&](const char *m) {
    g_create_error = m;
    mahi_batch_destroy(b);
    return MAHI_EDEVICE;
  };
  if (hipSetDevice(b->device) != hipSuccess) return bad("set device");
  if (hip_stream) {
    b->root = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&b->root, hipStreamNonBlocking) != hipSuccess) return bad("stream creation failed");
    b->own_root = true;
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) return bad("event creation failed");
  b->joins.assign(n_ctx, nullptr);
  for (auto &e : b->joins)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return bad("event creation failed");
  if (b->packed) {
    const std::string e = packed_setup(b, maxa, maxf);
    if (!e.empty()) {
      g_create_error = e;
      mahi_batch_destroy(b);
      return MAHI_EDEVICE;
    }
  }
  *out = b;
  return MAHI_OK;
}

mahi_status mahi_batch_eval(mahi_batch *b, const mahi_eval_args *args) {
  if (!b) return MAHI_EINVAL;
  if (!args) return b->fail(MAHI_EINVAL, "args is NULL");
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    const mahi_ctx *ctx = b->ctxs[i];
    if (!args[i].xyz) return b->fail(MAHI_EINVAL, "args[" + std::to_string(i) + "].xyz is NULL");
    if (args[i].flags != MAHI_DEVICE_IO) return b->fail(MAHI_EINVAL, "batched evaluation needs MAHI_DEVICE_IO");
    if (!ctx->lambda_set) return b->fail(MAHI_ESTATE, "system " + std::to_string(i) + ": lambda-tilde not set");
    if (ctx->prof_max > 0) return b->fail(MAHI_ESTATE, "system " + std::to_string(i) + ": stage profiling is open");
  }
  BATCH_TRY(hipSetDevice(b->device), "set device");
  if (b->packed) {
    const mahi_status st = packed_table(b, args);
    if (st != MAHI_OK) return st;
    if (!b->use_graph) {
      launch_packed(b->pp, b->root);
      BATCH_TRY(hipGetLastError(), "packed launch");
      return MAHI_OK;
    }
    if (!b->exec) {
      // one stream, kernel launches only: capture them once per set of arguments
      BATCH_TRY(hipStreamBeginCapture(b->root, hipStreamCaptureModeThreadLocal), "begin capture");
      launch_packed(b->pp, b->root);
      const hipError_t el = hipGetLastError();
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(b->root, &g);
      if (el != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return b->fail(MAHI_EDEVICE, std::string("capture: ") + hip_msg(el != hipSuccess ? el : e));
      }
      b->graph = g;
      const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        batch_drop_graph(b);
        return b->fail(MAHI_EDEVICE, std::string("graph instantiate: ") + hip_msg(ei));
      }
    }
    BATCH_TRY(hipGraphLaunch(b->exec, b->root), "graph launch");
    return MAHI_OK;
  }
  if (!b->use_graph) return batch_issue(b, args);
  bool same = b->exec != nullptr && b->captured.size() == b->ctxs.size();
  for (size_t i = 0; same && i < b->ctxs.size(); ++i) same = same_args(args[i], b->captured[i]);
  if (!same) {
    batch_drop_graph(b);
    BATCH_TRY(hipStreamBeginCapture(b->root, hipStreamCaptureModeRelaxed), "begin capture");
    const mahi_status st = batch_issue(b, args);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->root, &g);
    if (st != MAHI_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return b->fail(MAHI_EDEVICE, std::string("end capture: ") + hip_msg(e));
    b->graph = g;
    const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      batch_drop_graph(b);
      return b->fail(MAHI_EDEVICE, std::string("graph instantiate: ") + hip_msg(ei));
    }
    b->captured.assign(args, args + b->ctxs.size());
  }
  BATCH_TRY(hipGraphLaunch(b->exec, b->root), "graph launch");
  return MAHI_OK;
}

void mahi_batch_destroy(mahi_batch *b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->root) (void)hipStreamSynchronize(b->root);
  batch_drop_graph(b);
  for (auto &d : b->bufs) (void)hipFree(d.p);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (auto &e : b->joins)
    if (e) (void)hipEventDestroy(e);
  if (b->own_root && b->root) (void)hipStreamDestroy(b->root);
  delete b;
}

const char *mahi_batch_last_error(const mahi_batch *b) {
  if (!b) return g_create_error.c_str();
  return b->err.c_str();
}

mahi_status mahi_tune(mahi_ctx *ctx, const void *xyz, int reps, int *m2l_ranges, int *p2p_targets) {
  if (!ctx) return MAHI_EINVAL;
  if (!xyz) return ctx->fail(MAHI_EINVAL, "xyz is NULL");
  if (reps < 1 || reps > 1000) return ctx->fail(MAHI_ERANGE, "reps must be in 1..1000");
  if (!ctx->lambda_set) return ctx->fail(MAHI_ESTATE, "lambda-tilde not set");
  if (ctx->prof_max > 0) return ctx->fail(MAHI_ESTATE, "stage profiling is open");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  // the context's own output buffers; forces and dE/dlambda-tilde as in a full evaluation
  mahi_eval_args a{};
  a.xyz = xyz;
  a.forces = ctx->F;
  a.energy = ctx->E;
  a.dvdl = ctx->M > 0 ? ctx->dvdl : nullptr;
  a.flags = MAHI_DEVICE_IO;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return ctx->fail(MAHI_EDEVICE, "event");
  }
  auto timed = [&](float &ms) -> mahi_status {
    mahi_status st = ctx->prec == 32 ? eval_impl<float>(ctx, &a) : eval_impl<double>(ctx, &a);  // warm-up
    if (st != MAHI_OK) return st;
    if (hipEventRecord(e0, ctx->stream) != hipSuccess) return ctx->fail(MAHI_EDEVICE, "event record");
    for (int r = 0; r < reps && st == MAHI_OK; ++r)
      st = ctx->prec == 32 ? eval_impl<float>(ctx, &a) : eval_impl<double>(ctx, &a);
    if (st != MAHI_OK) return st;
    if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return ctx->fail(MAHI_EDEVICE, "event timing");
    return MAHI_OK;
  };
  mahi_status st = MAHI_OK;
  // float32 M2L: operator ranges of the main launch (the partial-sum array holds kM2LMaxSplit)
  if (ctx->prec == 32 && ctx->plan32.ntiles > 0) {
    const int keep = ctx->plan32.nsplit;
    int best = keep;
    float best_ms = 1e30f;
    for (int ns : {1, 2, 3, 4, 5, 6, 8}) {
      if (ns > kM2LMaxSplit) continue;
      ctx->plan32.nsplit = ns;
      float ms = 0.f;
      st = timed(ms);
      if (st != MAHI_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = ns;
      }
    }
    ctx->plan32.nsplit = st == MAHI_OK ? best : keep;
  }
  // near field: most targets per lane
  if (st == MAHI_OK) {
    const int keep = ctx->p2p_mmax;
    int best = keep;
    float best_ms = 1e30f;
    for (int mm = 1; mm <= 3 && st == MAHI_OK; ++mm) {
      ctx->p2p_mmax = mm;
      float ms = 0.f;
      st = timed(ms);
      if (st == MAHI_OK && ms < best_ms) {
        best_ms = ms;
        best = mm;
      }
    }
    ctx->p2p_mmax = st == MAHI_OK ? best : keep;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != MAHI_OK) return st;
  if (m2l_ranges) *m2l_ranges = ctx->prec == 32 ? ctx->plan32.nsplit : 0;
  if (p2p_targets) *p2p_targets = ctx->p2p_mmax;
  return MAHI_OK;
}

mahi_status mahi_autotune(int periodic, double edge, int64_t n_atoms, int precision, double target,
                          double site_extent, int *order, int *depth) {
  if (!order || !depth) return MAHI_EINVAL;
  if (periodic != 0 && periodic != 1) return MAHI_EINVAL;
  if (!(is_fin(edge) && edge > 0)) return MAHI_EINVAL;
  if (precision != 32 && precision != 64) return MAHI_EINVAL;
  if (!(is_fin(target) && target > 0) || !is_fin(site_extent)) return MAHI_EINVAL;
  if (n_atoms < 1 || n_atoms > (int64_t)0x7fffffff - 1) return MAHI_ERANGE;
  if (target < (precision == 32 ? 2e-5 : 2e-8)) return MAHI_ERANGE;
  // error envelope: the largest relative RMS error of forces and
  // dE/dlambda-tilde over water boxes of 900..60,000 atoms at their tuned
  // depths, against Ewald sums, with a margin.  Sites within 1 nm (the
  // clustered sites span ~0.6 nm) keep their intra-site pairs in the near
  // field; sites spread over the box (or of unknown extent) put them in the
  // far field, where the correction inherits the truncation error.
  const bool spread = site_extent < 0.0 || site_extent > 1.0;
  const double e8 = spread ? 5.0e-4 : 1.75e-4, f = spread ? 0.40 : 0.41;
  int p = 0;
  for (int c = 1; c <= kMaxOrder && !p; ++c)
    if (e8 * std::pow(f, c - 8) <= target) p = c;
  if (!p) return MAHI_ERANGE;
  // seconds per unit, from the 1,004,296-atom depth-5 order-8 stage times
  const bool f32 = precision == 32;
  const double c_pair = f32 ? 6.6e-13 : 2.2e-12;                  // ordered near-field pair
  const double kk = (p + 1.0) * (p + 1.0) / 81.0;
  const double c_tr = (f32 ? 1.5e-10 : 4.4e-10) * kk * kk;       // one M2L translation, dense (p+1)^2 squared
  const double c_leaf = 2.0e-9 * kk;                               // P2M / L2P / block overhead per leaf
  const double c_lvl = 2.0e-5;                                     // launch latency per tree level
  // one leaf's near field runs in one 64-lane block: with few, crowded leaves
  // the evaluation waits on that block (seconds per pair of one leaf, measured
  // on lone blocks of 3k..24k-atom systems at depths 1..2)
  const double c_blk = f32 ? 1.05e-9 : 3.6e-9;
  const double n = (double)n_atoms;
  double best = 1e300;
  int bd = 0;
  for (int d = 0; d <= 7; ++d) {
    const double leaves = std::ldexp(1.0, 3 * d);
    const double nb = periodic ? 27.0 : std::min(27.0, leaves);
    const double pairs = n * nb * n / leaves;
    double tr = 0.0;
    for (int l = periodic ? 1 : 2; l <= d; ++l) tr += 189.0 * std::ldexp(1.0, 3 * l);
    const double per_leaf = n / leaves;
    const double t = c_pair * pairs + c_blk * nb * per_leaf * per_leaf + c_tr * tr + c_leaf * leaves + c_lvl * d;
    if (t < best) {
      best = t;
      bd = d;
    }
  }
  *order = p;
  *depth = bd;
  (void)edge;
  return MAHI_OK;
}

mahi_status mahi_host_selftest(int order, double *max_rel_err) {
  if (!max_rel_err) return MAHI_EINVAL;
  if (order < 1 || order > kMaxOrder) return MAHI_ERANGE;
  *max_rel_err = host_selftest(order);
  return MAHI_OK;
}

mahi_status mahi_device_selftest(int precision, double *max_rel_err) {
  if (!max_rel_err || (precision != 32 && precision != 64)) return MAHI_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MAHI_EDEVICE;
  const int rows = precision == 32 ? 96 : 48, kk = 84;
  std::mt19937_64 rng(5);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<double> A((size_t)kk * rows), B((size_t)kk * 64), C((size_t)rows * 64, 0.0);
  for (auto &v : A) v = U(rng);
  for (auto &v : B) v = U(rng);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < 64; ++c)
      for (int k = 0; k < kk; ++k) C[(size_t)r * 64 + c] += A[(size_t)k * rows + r] * B[(size_t)k * 64 + c];
  // probe: 0 the tile code of the generic translation kernels (32x32x2 float32,
  // 16x16x4 float64), 1 the float32 16x16x4 tile of the M2L kernel for orders up to 8
  auto run = [&](auto zero, int probe) -> mahi_status {
    using T = decltype(zero);
    std::vector<T> a(A.begin(), A.end()), b(B.begin(), B.end()), c((size_t)rows * 64);
    T *da = nullptr, *db = nullptr, *dc = nullptr;
    if (hipMalloc(&da, sizeof(T) * a.size()) != hipSuccess || hipMalloc(&db, sizeof(T) * b.size()) != hipSuccess ||
        hipMalloc(&dc, sizeof(T) * c.size()) != hipSuccess)
      return MAHI_ENOMEM;
    (void)hipMemcpy(da, a.data(), sizeof(T) * a.size(), hipMemcpyHostToDevice);
    (void)hipMemcpy(db, b.data(), sizeof(T) * b.size(), hipMemcpyHostToDevice);
    if constexpr (sizeof(T) == sizeof(float)) {
      if (probe == 1) launch_mfma16_probe(da, db, dc, rows, kk, nullptr);
      else launch_mfma_probe<T>(da, db, dc, rows, kk, nullptr);
    } else {
      launch_mfma_probe<T>(da, db, dc, rows, kk, nullptr);
    }
    hipError_t e = hipDeviceSynchronize();
    (void)hipMemcpy(c.data(), dc, sizeof(T) * c.size(), hipMemcpyDeviceToHost);
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(dc);
    if (e != hipSuccess) return MAHI_EDEVICE;
    double worst = 0.0, nrm = 0.0;
    for (size_t i = 0; i < c.size(); ++i) {
      worst = std::max(worst, std::fabs((double)c[i] - C[i]));
      nrm = std::max(nrm, std::fabs(C[i]));
    }
    *max_rel_err = std::max(*max_rel_err, worst / nrm);
    return MAHI_OK;
  };
  *max_rel_err = 0.0;
  if (precision == 64) return run(0.0, 0);
  const mahi_status st = run(0.0f, 0);
  return st != MAHI_OK ? st : run(0.0f, 1);
}

}  // extern "C"
