// Host side of libmcr: handle, workspaces, argument validation, the drivers
// of Algorithm 1 and the FP64 diagnostics. Implements include/mcr.h.
#include "mcr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "mcr_kernels.h"
#include "mcr_joseph_tiled.h"
#include "mcr_grad.h"
#include "mcr_register.h"

using namespace mcr;

namespace {

thread_local std::string g_err;

mcr_status fail(mcr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_OK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? MCR_ERR_NOMEM : MCR_ERR_HIP, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                       \
  } while (0)

#define LAUNCH_OK() HIP_OK(hipGetLastError())

#define STATUS_OK(expr)           \
  do {                            \
    mcr_status s_ = (expr);       \
    if (s_ != MCR_OK) return s_;  \
  } while (0)

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

constexpr int kFwdKA = 8, kFwdJD = 32, kFwdWL = 128;  // tiled forward: angles, bins, LDS row
constexpr int kMaxShares = 16;                          // tiled adjoint: angle shares
constexpr double kMaxBlurSigma = 32.0;  // widest scale-space Gaussian of the dense registration (px)
constexpr int kMaxBlurRadius = 96;      // int(3 kMaxBlurSigma + 0.5)
constexpr int kMaxLevels = 16;          // scale-space levels per dense registration


// Work tables of a quarter-turn forward (k_joseph_fwd_quad<MODE, NP>): the
// line-sheared schedule over its primary angles, XCD-ordered pieces, and per
// paired angle subset the ranges of pieces and multi-piece units.
struct QuadTables {
  int4* chunks = nullptr;
  int4* pieces = nullptr;
  int4* units = nullptr;
  int4* bands = nullptr;
  float* part = nullptr;  // [slots][part_floats]
  int* multi = nullptr;
  int npieces = 0, nmulti = 0;
  long part_floats = 0;
  std::vector<int2> sub;        // paired subsets: (first piece, pieces) per subset
  std::vector<int2> sub_multi;  // paired subsets: (first multi-piece unit entry, entries) per subset
};

// Per-precision workspace and tables.
template <typename T>
struct Work {
  bool ready = false;
  AngleT<T>* ang = nullptr;          // [n_angles]
  AngleFx* angfx = nullptr;          // [n_angles] (float workspace only)
  GateMotion<T>* motion = nullptr;   // [N + 1]; entry N is the identity
  GateScalars<T>* scalars = nullptr; // [N]
  GatePtrs<T>* ptrs = nullptr;       // [N]
  T* wP = nullptr;                   // [N][padded]
  T* wTP = nullptr;                  // [N][padded]
  T* wQ = nullptr;                   // [N][7][padded] planes P_1..P_3 (even n and n_angles), Q_0..Q_3 (and
                                     // n_angles a multiple of 4) of the quarter-turn forwards (float)
  T* bP = nullptr;                   // [N][padded]
  T* dy = nullptr;                   // [N][sino]
  T* img = nullptr;                  // [n*n] scratch
  T* img2 = nullptr;                 // [n*n] scratch
  // host staging for scalars and pointers, uploaded when they change
  void* pin = nullptr;
  size_t pin_bytes = 0;
  hipEvent_t pin_ev = nullptr;
  bool pin_recorded = false;
  std::vector<char> last;
  std::vector<GateScalars<T>> sc_host;  // last tables handed to upload_params
  std::vector<GatePtrs<T>> pt_host;
  int sc_base = 0;                      // first scalar entry the launches use (angle subset s: s N)
  int sc_cap = 0;                       // scalar entries allocated
};

}  // namespace

struct mcr_handle {
  mcr_geometry geo{};
  int N = 0;
  int nslots = 0;  // workspace slots: gates one launch may cover (N, or the slices of a batch)
  mcr_dtype dtype = MCR_F32;
  hipStream_t stream = nullptr;
  int pitch = 0;
  long padded = 0;   // elements of one padded image
  long sino = 0;     // elements of one sinogram
  std::vector<mcr_motion> motion;  // host copy (field pointers not kept)
  std::vector<int> radius;         // per gate
  float* fieldP = nullptr;         // [N][2][padded]
  short2* centres = nullptr;       // [N][n][n]
  bool any_field = false;
  Work<float> wf;
  Work<double> wd;
  double* red_partial = nullptr;   // [kRedBlocks]
  double* red_out = nullptr;       // [64] result slots
  double* red_host = nullptr;      // pinned [64]
  int* need = nullptr;             // window verification
  double* mgrad_partial = nullptr; // [ceil(n/16)^2][3] motion-gradient partial sums
  void* mot_pin = nullptr;         // pinned staging of the motion tables (mcr_set_rigid_params)
  hipEvent_t mot_ev = nullptr;
  bool mot_recorded = false;
  std::vector<void*> allocs;
  // float32 projector pair: kernel variants (chosen by mcr_autotune)
  struct Tune {
    int fwd = 3;     // 0 one thread per ray, 1 LDS-tiled (8 angles x 32 bins), 2 the same with a host band
                     // schedule, 3 line-sheared bands (16 angles x 32 bins, two rays per thread), 4 the
                     // line-sheared quarter-turn forward (four rays per crossing)
    int adj_px = 4;  // 0 one thread per pixel; 1, 2, 4, 8 pixels per thread (LDS-tiled)
    int adj_s = 4;   // angle shares per pixel tile (LDS-tiled adjoint)
  } tune;
  bool fwd_lds_ok = false;         // every band window of the tiled forward fits in LDS
  int2* chunks = nullptr;          // angle chunks of the tiled forward
  int nchunks = 0;
  int4* sched_chunks = nullptr;    // scheduled forward: (k0, count, shear, -) per chunk
  int2* sched_blocks = nullptr;    // (first band, bands) per (chunk, detector tile)
  int4* sched_bands = nullptr;     // (L0, lines, window start, window width)
  int sched_nchunks = 0;
  bool sched_ok = false;
  int4* shear_chunks = nullptr;    // line-sheared forward: (k0, count, Bm low, Bm high) per chunk
  int4* shear_pieces = nullptr;    // (first band, bands, unit, piece) per block
  int4* shear_units = nullptr;     // (chunk, detector tile, pieces, partial-sum offset) per unit
  int4* shear_bands = nullptr;     // (L0, lines, window start, log2 of the LDS line pitch)
  float* shear_part = nullptr;     // [slots][part_floats] partial ray sums of multi-piece units
  int* shear_multi = nullptr;      // units cut into several pieces
  int shear_npieces = 0, shear_nmulti = 0;
  std::vector<int2> shear_sub;        // per angle subset: (first piece, pieces)
  std::vector<int2> shear_sub_multi;  // per angle subset: (first multi-piece unit entry, entries)
  // quarter-turn forwards: qt[0] four planes (variant 4, also per paired
  // angle subset), qt[1] eight planes (variant 5, all angles)
  QuadTables qt[2];
  // angle subsets (mcr_set_subsets, mcr_set_subset_partition): subset s holds
  // the angles of sub[s], one range or (paired) a range and its partner range
  int M = 1;
  bool sub_paired = false;
  std::vector<AngleRanges> sub;
  long shear_part_floats = 0;
  float* parts = nullptr;          // [kMaxShares][N][n*n] partial backprojections
  // affine registration scratch (allocated on first use)
  void* reg_g = nullptr;           // [2][n*n] field gradient planes (handle dtype)
  double* reg_partial = nullptr;   // [kRedBlocks][6] moment partials
  float* reg_field = nullptr;      // [2][n*n] the result field, unpadded
  double* reg_dense = nullptr;     // [4][2][n*n] dense registration: u, g, trial u, trial g (FP64)
  double* reg_blur = nullptr;      // [3][n*n] smoothed reference, target and a pass in between (handle dtype)
  double* reg_w = nullptr;         // [2 kMaxBlurRadius + 1] Gaussian weights
  // batched SPDHG (mcr_batch_create): S independent slices sharing the geometry
  struct Batch {
    int S = 0;                        // 0: not a batch handle
    std::vector<int> ng, off;         // gates per slice, first global gate of each slice
    int tmax = 0;                     // largest gate count = number of rounds
    std::vector<int> nact;            // slots of round t
    std::vector<int2> items;          // (slice, iteration) of every slot, round after round
    std::vector<int> round_off;       // first item of each round
    SlotInfo* slots = nullptr;        // device [tmax][S]
    void* tc = nullptr;               // device [S][2] (tau, c_x) in the handle's dtype
    void* pin = nullptr;              // pinned staging of slots + tc
    size_t pin_bytes = 0;
    hipEvent_t pin_ev = nullptr;
    bool pin_recorded = false;
    hipStream_t gstream = nullptr;    // stream the epoch graph runs on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[3] = {nullptr, nullptr, nullptr};  // x, z, zbar baked into the graph
    unsigned long gen = 0;            // handle's config_gen when the graph was captured
  } batch;
  // bumped whenever a choice that a captured launch sequence bakes in changes
  // (projector variants, gather-window radii)
  unsigned long config_gen = 0;
  // kernel timing
  bool prof = false;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> spare;
};

namespace {

mcr_status dmalloc(mcr_handle* h, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes < 256 ? 256 : bytes);
  if (e != hipSuccess) return fail(MCR_ERR_NOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  h->allocs.push_back(*p);
  HIP_OK(hipMemsetAsync(*p, 0, bytes < 256 ? 256 : bytes, h->stream));
  return MCR_OK;
}

hipEvent_t prof_event(mcr_handle* h) {
  if (!h->spare.empty()) {
    hipEvent_t e = h->spare.back();
    h->spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches made while alive with events when timing is enabled.
struct Timed {
  mcr_handle* h;
  int cls;
  hipEvent_t a = nullptr;
  Timed(mcr_handle* hh, int c) : h(hh), cls(c) {
    if (h->prof && h->recs.size() < 200000) {
      a = prof_event(h);
      if (a && hipEventRecord(a, h->stream) != hipSuccess) a = nullptr;
    }
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = prof_event(h);
    if (b && hipEventRecord(b, h->stream) == hipSuccess) {
      h->recs.push_back({cls, a, b});
    } else {
      h->spare.push_back(a);
      if (b) h->spare.push_back(b);
    }
  }
};

template <typename T>
Work<T>& work(mcr_handle* h);
template <>
Work<float>& work<float>(mcr_handle* h) { return h->wf; }
template <>
Work<double>& work<double>(mcr_handle* h) { return h->wd; }

template <typename T>
Geo<T> geo_of(const mcr_handle* h) {
  Geo<T> g;
  g.n = h->geo.n;
  g.na = h->geo.n_angles;
  g.nd = h->geo.n_det;
  g.pitch = h->pitch;
  g.hc = T((h->geo.n - 1) / 2.0);
  g.jc = T((h->geo.n_det - 1) / 2.0);
  return g;
}

// Joseph constants per angle in FP64, rounded once to T. The stepping axis is
// decided by the integer rule on k so that every precision uses the same matrix.
template <typename T>
std::vector<AngleT<T>> angle_table(int na) {
  std::vector<AngleT<T>> v(na);
  for (int k = 0; k < na; ++k) {
    const double th = M_PI * k / na;
    const double cs = std::cos(th), sn = std::sin(th);
    const bool rows = (4L * k <= na) || (4L * k >= 3L * na);
    AngleT<T> a{};
    if (rows) {
      a.a = T(1.0 / cs);
      a.beta = T(-sn / cs);
      a.ia = T(cs);
      a.ds = T(1.0 / std::fabs(cs));
    } else {
      a.a = T(1.0 / sn);
      a.beta = T(-cs / sn);
      a.ia = T(sn);
      a.ds = T(1.0 / std::fabs(sn));
    }
    a.rows = rows ? 1 : 0;
    v[k] = a;
  }
  return v;
}

template <typename T>
GateMotion<T> gate_motion(const mcr_handle* h, int gate) {
  GateMotion<T> m{};
  const double hc = (h->geo.n - 1) / 2.0;
  if (gate >= h->N) return m;  // the identity entry
  const mcr_motion& mo = h->motion[gate];
  m.kind = mo.kind;
  m.radius = h->radius[gate];
  if (mo.kind == MCR_MOTION_RIGID) {
    const double phi = mo.rigid[0];
    const double c = std::cos(phi), s = std::sin(phi);
    const double sh = std::sin(0.5 * phi);
    m.cm1 = T(-2.0 * sh * sh);  // cos - 1 without cancellation
    m.sn = T(s);
    m.tx = T(mo.rigid[1]);
    m.ty = T(mo.rigid[2]);
    m.i00 = T(c);
    m.i01 = T(s);
    m.i10 = T(-s);
    m.i11 = T(c);
    m.bx = T(hc + mo.rigid[1]);
    m.by = T(hc + mo.rigid[2]);
  }
  return m;
}

// Fixed-point constants of the float32 projector pair (see AngleFx).
std::vector<AngleFx> angle_table_fx(int n, int na, int nd) {
  std::vector<AngleFx> v(na);
  const double hc = (n - 1) / 2.0, jc = (nd - 1) / 2.0, one = 4294967296.0;
  for (int k = 0; k < na; ++k) {
    const double th = M_PI * k / na;
    const double cs = std::cos(th), sn = std::sin(th);
    const bool rows = (4L * k <= na) || (4L * k >= 3L * na);
    const double a = rows ? 1.0 / cs : 1.0 / sn;
    const double beta = rows ? -sn / cs : -cs / sn;
    const double c0 = hc - jc * a - hc * beta;  // cf(j, L) = c0 + j a + L beta
    const double ia = 1.0 / a;
    AngleFx f{};
    f.C0 = std::llround(c0 * one);
    f.A = std::llround(a * one);
    f.B = std::llround(beta * one);
    f.U0 = std::llround(-c0 * ia * one);
    f.P = std::llround(ia * one);
    f.Q = std::llround(-beta * ia * one);
    f.RS = rows ? f.P : f.Q;
    f.a = float(a);
    f.beta = float(beta);
    f.absa = float(std::fabs(a));
    f.oma = float(1.0 - std::fabs(a));
    f.ds = float(std::fabs(a));
    f.rows = rows ? 1 : 0;
    f.na32 = float(-std::fabs(a) / one);
    f.pa32 = float(std::fabs(a) / one);
    v[k] = f;
  }
  return v;
}

template <typename T>
mcr_status upload_motion(mcr_handle* h) {
  Work<T>& w = work<T>(h);
  std::vector<GateMotion<T>> gm(h->N + 1);
  for (int i = 0; i <= h->N; ++i) gm[i] = gate_motion<T>(h, i);
  HIP_OK(hipMemcpyAsync(w.motion, gm.data(), sizeof(GateMotion<T>) * gm.size(), hipMemcpyHostToDevice,
                        h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  return MCR_OK;
}

// Runs of at most ka consecutive angles of one stepping type.
std::vector<int2> angle_chunks(const std::vector<AngleFx>& af, int ka) {
  std::vector<int2> ch;
  int k = 0;
  const int na = (int)af.size();
  while (k < na) {
    int e = k + 1;
    while (e < na && e - k < ka && af[e].rows == af[k].rows) ++e;
    ch.push_back(make_int2(k, e - k));
    k = e;
  }
  return ch;
}

// The tiled forward stages, per band, the sheared window spanned by the
// crossings of its corner rays. A single line's window is widest on the first
// or the last image line (max - min of affine functions is convex); check that
// it fits the LDS row for every chunk and detector tile.
bool tiled_windows_fit(const mcr_handle* h, const std::vector<AngleFx>& af, const std::vector<int2>& ch) {
  const int nd = h->geo.n_det, n = h->geo.n;
  for (const int2& c : ch) {
    for (int j0 = 0; j0 < nd; j0 += kFwdJD) {
      const int j1 = std::min(j0 + kFwdJD - 1, nd - 1);
      for (int L : {0, n - 1}) {
        long long lo = LLONG_MAX, hi = LLONG_MIN;
        for (int a = 0; a < c.y; ++a) {
          const AngleFx& A = af[c.x + a];
          for (int j : {j0, j1}) {
            const long long v = (A.C0 + (long long)j * A.A + (long long)L * A.B) >> 32;
            lo = std::min(lo, v);
            hi = std::max(hi, v);
          }
        }
        if (hi - lo + 3 > kFwdWL) return false;
      }
    }
  }
  return true;
}

// Band schedule of the scheduled tiled forward (see k_joseph_fwd_sched): for
// each chunk of angles and tile of bins, the lines any of its rays crosses
// inside (-1, n), cut into bands of at most kFwdMaxBand lines whose sheared
// windows (over the corner rays, exact integer arithmetic) fit kFwdWL columns.
struct Schedule {
  std::vector<int4> chunks;
  std::vector<int2> blocks;
  std::vector<int4> bands;
  bool ok = true;
  // line-sheared forward only: work pieces and units (see k_joseph_fwd_shear)
  std::vector<int4> pieces;  // (first band, bands, unit, piece index)
  std::vector<int4> units;   // (chunk, detector tile, pieces P, offset of the unit's partial sums)
  std::vector<int> multi;    // units with P > 1
  long part_floats = 0;      // partial sums per gate slot
  std::vector<int2> sub_pieces, sub_multi;  // per angle subset: (first, count) of pieces / multi entries
};

// Lines [L_lo, L_hi] on which some ray of angles [k0, k0 + cnt) and bins
// [jf, jl] crosses inside (-1, n), widened by a margin of 2; empty if L_lo > L_hi.
void block_lines(int n, int nd, const std::vector<AngleFx>& af, int k0, int cnt, int jf, int jl, int& L_lo,
                 int& L_hi) {
  const double hc = (n - 1) / 2.0, jc = (nd - 1) / 2.0;
  double lo = n, hi = -1;
  for (int a = 0; a < cnt; ++a) {
    const AngleFx& A = af[k0 + a];
    const double a_ = double(A.A) / 4294967296.0, b_ = double(A.B) / 4294967296.0;
    const double ta_f = (jf - jc) * a_ + hc, ta_l = (jl - jc) * a_ + hc;  // crossings on the centre line
    if (std::fabs(b_) < 1e-12) {  // crossings do not move with the line
      if (std::max(ta_f, ta_l) > -1.0 && std::min(ta_f, ta_l) < n) {
        lo = 0;
        hi = n - 1;
      }
      continue;
    }
    for (double ta : {ta_f, ta_l}) {
      const double u1 = (-1.0 - ta) / b_ + hc, u2 = (n - ta) / b_ + hc;
      lo = std::min(lo, std::min(u1, u2));
      hi = std::max(hi, std::max(u1, u2));
    }
  }
  L_lo = std::max(0, (int)std::floor(std::max(lo, -4.0)) - 2);
  L_hi = std::min(n - 1, (int)std::ceil(std::min(hi, n + 4.0)) + 2);
}

// Bands of one block of the line-sheared forward (exact integer arithmetic on
// the kernel's constants): the window of band line l is shifted by
// o_l = floor(l Bm / 2^32). A band of BL lines with window width W is staged
// with a power-of-two line pitch P >= max(64, W) and needs BL * P <= kShCap
// entries; bands start at kShBL lines and are shortened until they fit.
// Returns false if a single line does not fit.
bool shear_tile_bands(int n, int nd, const std::vector<AngleFx>& af, int k0, int cnt, long long Bm, int jf, int jl,
                      int cap, std::vector<int4>& bands) {
  int L_lo, L_hi;
  block_lines(n, nd, af, k0, cnt, jf, jl, L_lo, L_hi);
  for (int L0 = L_lo; L0 <= L_hi;) {
    int bl = std::min(kShBL, L_hi - L0 + 1);
    int S0 = 0, lp = 6;
    for (;;) {
      long long vmin = LLONG_MAX, vmax = LLONG_MIN;
      for (int a = 0; a < cnt; ++a) {
        const AngleFx& A = af[k0 + a];
        for (int j : {jf, jl}) {
          const long long base = A.C0 + (long long)j * A.A + (long long)L0 * A.B;
          for (int l = 0; l < bl; ++l) {
            const long long v = ((base + (long long)l * A.B) >> 32) - (((long long)l * Bm) >> 32);
            vmin = std::min(vmin, v);
            vmax = std::max(vmax, v);
          }
        }
      }
      S0 = (int)vmin - 1;
      const long long W = vmax - vmin + 3;
      lp = 6;
      while ((1LL << lp) < W) ++lp;
      if ((long long)bl << lp <= cap) break;
      if (bl == 1) return false;
      bl = std::max(1, (int)(cap >> lp));
    }
    bands.push_back(make_int4(L0, bl, S0, lp));
    L0 += bl;
  }
  return true;
}

// Chunks of up to kShKA consecutive angles of each run (runs: consecutive
// angles of one stepping type and one angle subset, bounds: k_0 = 0 < ... <
// k_M = n_angles), halved where a line of some detector tile does not fit the
// window; detector tiles of kShJD bins cover bins [0, nbins); cap: staged
// entries per band; ppp: partial sums per piece.
Schedule build_shear_units(int n, int nd, int nbins, const std::vector<AngleFx>& af, const std::vector<int2>& runs,
                           const std::vector<int>& asub, int M, int cap, int ppp, int piece_lines) {
  Schedule S;
  const int ntiles = (nbins + kShJD - 1) / kShJD;
  for (const int2& run : runs) {
    for (int k0 = run.x; k0 < run.x + run.y;) {
      int cnt = std::min(kShKA, run.x + run.y - k0);
      std::vector<int2> blocks;
      std::vector<int4> bands;
      for (;;) {
        const long long Bm = af[k0 + cnt / 2].B;
        blocks.clear();
        bands.clear();
        bool fit = true;
        for (int t = 0; t < ntiles && fit; ++t) {
          const int jf = t * kShJD, jl = std::min(jf + kShJD - 1, nbins - 1);
          const int first = (int)(S.bands.size() + bands.size());
          fit = shear_tile_bands(n, nd, af, k0, cnt, Bm, jf, jl, cap, bands);
          blocks.push_back(make_int2(first, (int)(S.bands.size() + bands.size()) - first));
        }
        if (fit) {
          S.chunks.push_back(make_int4(k0, cnt, (int)(unsigned)(Bm & 0xffffffffLL), (int)(Bm >> 32)));
          break;
        }
        if (cnt == 1) {
          S.ok = false;
          return S;
        }
        cnt = (cnt + 1) / 2;
      }
      S.blocks.insert(S.blocks.end(), blocks.begin(), blocks.end());
      S.bands.insert(S.bands.end(), bands.begin(), bands.end());
      k0 += cnt;
    }
  }
  // cut every (chunk, tile) unit into pieces of about piece_lines lines so
  // that the blocks carry similar work; pieces of one unit are numbered in
  // line order and their partial sums are added in that order
  for (int c = 0; c < (int)S.chunks.size(); ++c) {
    for (int t = 0; t < ntiles; ++t) {
      const int u = c * ntiles + t;
      const int2 bl = S.blocks[u];
      int b0 = bl.x, lines = 0, pc = 0;
      for (int b = bl.x; b < bl.x + bl.y; ++b) {
        if (b > b0 && lines + S.bands[b].y > piece_lines) {
          S.pieces.push_back(make_int4(b0, b - b0, u, pc++));
          b0 = b;
          lines = 0;
        }
        lines += S.bands[b].y;
      }
      S.pieces.push_back(make_int4(b0, bl.x + bl.y - b0, u, pc++));
      if (pc > 1) S.multi.push_back((int)S.units.size());
      S.units.push_back(make_int4(c, t, pc, (int)S.part_floats));
      if (pc > 1) S.part_floats += (long)pc * ppp;
    }
  }
  // pieces and multi-piece units come in chunk order and the runs in subset
  // order, so each subset's are contiguous
  S.sub_pieces.assign(M, make_int2(0, 0));
  S.sub_multi.assign(M, make_int2(0, 0));
  auto subset_of = [&](int unit) { return asub[S.chunks[S.units[unit].x].x]; };
  for (int q = 0; q < (int)S.pieces.size(); ++q) {
    int2& r = S.sub_pieces[subset_of(S.pieces[q].z)];
    if (r.y == 0) r.x = q;
    ++r.y;
  }
  for (int q = 0; q < (int)S.multi.size(); ++q) {
    int2& r = S.sub_multi[subset_of(S.multi[q])];
    if (r.y == 0) r.x = q;
    ++r.y;
  }
  return S;
}

// Runs of `runs` cut where the subset changes, in subset order (stable).
std::vector<int2> cut_runs(const std::vector<int2>& runs, const std::vector<int>& asub) {
  std::vector<int2> out;
  for (const int2& r : runs) {
    int k = r.x;
    for (int e = r.x + 1; e <= r.x + r.y; ++e) {
      if (e == r.x + r.y || asub[e] != asub[k]) {
        out.push_back(make_int2(k, e - k));
        k = e;
      }
    }
  }
  std::stable_sort(out.begin(), out.end(), [&](const int2& a, const int2& b) { return asub[a.x] < asub[b.x]; });
  return out;
}

// Line-sheared forward over all angles: runs of one stepping type and one
// subset (asub: the subset of every angle), in subset order.
Schedule build_shear_schedule(int n, int nd, const std::vector<AngleFx>& af, const std::vector<int>& asub, int M) {
  return build_shear_units(n, nd, nd, af, cut_runs(angle_chunks(af, INT_MAX), asub), asub, M, kShCap, 2 * 256,
                           kShPieceLines);
}

// Quarter-turn forward: the primary angles are the row-stepping ones
// (4k <= n_angles or 4k >= 3 n_angles), without k = 3 n_angles / 4 (the
// partner of k = n_angles / 4); with n_angles even each pair {k, k +- n_angles/2}
// holds exactly one primary angle. Bins [0, ceil(n_det / 2)).
// asub: the subset of every angle, the same for an angle and its partner
// (paired subsets, or one subset); runs cut by subset, in subset order.
// NP = 8 (n_angles a multiple of 4): the primary angles are k = 0 ..
// n_angles/4, each also serving the transposed image's rays.
Schedule build_quad_schedule(int n, int nd, const std::vector<AngleFx>& af, const std::vector<int>& asub, int M,
                             int NP = 4) {
  const int na = (int)af.size();
  std::vector<int2> runs;
  const int a_end = na / 4 + 1;                  // k <= floor(na / 4)
  const int b_beg = (3 * na + 3) / 4 + (na % 4 == 0 ? 1 : 0);
  if (a_end > 0) runs.push_back(make_int2(0, std::min(a_end, na)));
  if (NP == 4 && b_beg < na) runs.push_back(make_int2(b_beg, na - b_beg));
  return build_shear_units(n, nd, (nd + 1) / 2, af, cut_runs(runs, asub), asub, M, kQuCap, 2 * NP * 256,
                           NP == 8 ? kOcPieceLines : kQuPieceLines);
}

Schedule build_schedule(int n, int nd, const std::vector<AngleFx>& af, int ka, int jd, int wl) {
  Schedule S;
  const std::vector<int2> ch = angle_chunks(af, ka);
  const int ntiles = (nd + jd - 1) / jd;
  for (const int2& c : ch) {
    // the same shear the kernel applies: rint of the float slope of the middle angle
    const int m = (int)std::nearbyint(af[c.x + (c.y >> 1)].beta);
    S.chunks.push_back(make_int4(c.x, c.y, m, 0));
  }
  for (size_t ci = 0; ci < ch.size(); ++ci) {
    const int2 c = ch[ci];
    const int m = S.chunks[ci].z;
    for (int t = 0; t < ntiles; ++t) {
      const int jf = t * jd, jl = std::min(jf + jd - 1, nd - 1);
      int L_lo, L_hi;
      block_lines(n, nd, af, c.x, c.y, jf, jl, L_lo, L_hi);
      const int first = (int)S.bands.size();
      for (int L0 = L_lo; L0 <= L_hi;) {
        int bl = std::min(kFwdMaxBand, L_hi - L0 + 1);
        int S0 = 0, W = 0;
        for (;; bl = (bl + 1) / 2) {
          long long vmin = LLONG_MAX, vmax = LLONG_MIN;
          for (int a = 0; a < c.y; ++a) {
            const AngleFx& A = af[c.x + a];
            for (int j : {jf, jl}) {
              for (int l : {0, bl - 1}) {
                const long long v = ((A.C0 + (long long)j * A.A + (long long)(L0 + l) * A.B) >> 32) -
                                    (long long)l * m;
                vmin = std::min(vmin, v);
                vmax = std::max(vmax, v);
              }
            }
          }
          S0 = (int)vmin - 1;
          W = (int)(vmax - vmin) + 3;
          if (W <= wl || bl == 1) break;
        }
        if (W > wl) S.ok = false;
        S.bands.push_back(make_int4(L0, bl, S0, W));
        L0 += bl;
      }
      S.blocks.push_back(make_int2(first, (int)S.bands.size() - first));
    }
  }
  return S;
}

void dfree(mcr_handle* h, void* p) {
  if (!p) return;
  auto it = std::find(h->allocs.begin(), h->allocs.end(), p);
  if (it != h->allocs.end()) h->allocs.erase(it);
  (void)hipFree(p);
}

// The subset of every angle under the handle's partition.
std::vector<int> angle_subsets(const mcr_handle* h) {
  std::vector<int> asub(h->geo.n_angles, 0);
  for (int s = 0; s < (int)h->sub.size(); ++s) {
    const AngleRanges& r = h->sub[s];
    for (int k = r.ka; k < r.kb; ++k) asub[k] = s;
    for (int k = r.kc; k < r.kd; ++k) asub[k] = s;
  }
  return asub;
}

// (Re)builds the line-sheared forward's tables for the handle's angle subsets.
// Synchronises the stream (the previous tables may still be in use).
mcr_status upload_shear(mcr_handle* h, const std::vector<AngleFx>& af) {
  HIP_OK(hipStreamSynchronize(h->stream));
  for (void* p : {(void*)h->shear_chunks, (void*)h->shear_pieces, (void*)h->shear_units, (void*)h->shear_bands,
                  (void*)h->shear_part, (void*)h->shear_multi})
    dfree(h, p);
  h->shear_chunks = h->shear_pieces = h->shear_units = h->shear_bands = nullptr;
  h->shear_part = nullptr;
  h->shear_multi = nullptr;
  h->shear_npieces = h->shear_nmulti = 0;
  h->shear_sub.clear();
  h->shear_sub_multi.clear();
  const Schedule ss = build_shear_schedule(h->geo.n, h->geo.n_det, af, angle_subsets(h), h->M);
  if (!ss.ok) return MCR_OK;  // variant 3 unavailable on this geometry
  const int ns = h->nslots;
  h->shear_part_floats = ss.part_floats;
  STATUS_OK(dmalloc(h, (void**)&h->shear_chunks, sizeof(int4) * ss.chunks.size()));
  STATUS_OK(dmalloc(h, (void**)&h->shear_pieces, sizeof(int4) * ss.pieces.size()));
  STATUS_OK(dmalloc(h, (void**)&h->shear_units, sizeof(int4) * ss.units.size()));
  STATUS_OK(dmalloc(h, (void**)&h->shear_bands, sizeof(int4) * std::max<size_t>(1, ss.bands.size())));
  STATUS_OK(dmalloc(h, (void**)&h->shear_part, sizeof(float) * std::max<long>(1, ss.part_floats) * ns));
  STATUS_OK(dmalloc(h, (void**)&h->shear_multi, sizeof(int) * std::max<size_t>(1, ss.multi.size())));
  HIP_OK(hipMemcpyAsync(h->shear_chunks, ss.chunks.data(), sizeof(int4) * ss.chunks.size(), hipMemcpyHostToDevice,
                        h->stream));
  HIP_OK(hipMemcpyAsync(h->shear_pieces, ss.pieces.data(), sizeof(int4) * ss.pieces.size(), hipMemcpyHostToDevice,
                        h->stream));
  HIP_OK(hipMemcpyAsync(h->shear_units, ss.units.data(), sizeof(int4) * ss.units.size(), hipMemcpyHostToDevice,
                        h->stream));
  if (!ss.bands.empty())
    HIP_OK(hipMemcpyAsync(h->shear_bands, ss.bands.data(), sizeof(int4) * ss.bands.size(), hipMemcpyHostToDevice,
                          h->stream));
  if (!ss.multi.empty())
    HIP_OK(hipMemcpyAsync(h->shear_multi, ss.multi.data(), sizeof(int) * ss.multi.size(), hipMemcpyHostToDevice,
                          h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  h->shear_npieces = (int)ss.pieces.size();
  h->shear_nmulti = (int)ss.multi.size();
  h->shear_sub = ss.sub_pieces;
  h->shear_sub_multi = ss.sub_multi;
  return MCR_OK;
}

// Tables of the quarter-turn forwards (float handles with even n and
// n_angles): four planes over all angles and, with paired subsets, per
// subset; eight planes over all angles where n_angles is a multiple of 4.
// Rebuilding frees the previous tables (synchronises the stream).
mcr_status upload_quad_tables(mcr_handle* h, const std::vector<AngleFx>& af, int which) {
  QuadTables& qt = h->qt[which];
  const int NP = which ? 8 : 4;
  for (void* p : {(void*)qt.chunks, (void*)qt.pieces, (void*)qt.units, (void*)qt.bands, (void*)qt.part,
                  (void*)qt.multi})
    dfree(h, p);
  qt = QuadTables{};
  if (h->geo.n % 2 || h->geo.n_angles % (2 * NP / 4)) return MCR_OK;
  // the kernels address a padded plane with 32-bit byte offsets
  if (4L * h->padded >= (1L << 31)) return MCR_OK;
  // the subsets the four-plane kernels can serve: one, or paired ones; the
  // eight-plane kernels serve launches over all angles only
  const bool by_subset = NP == 4 && h->M > 1 && h->sub_paired;
  const std::vector<int> asub = by_subset ? angle_subsets(h) : std::vector<int>(h->geo.n_angles, 0);
  const int M = by_subset ? h->M : 1;
  Schedule qs = build_quad_schedule(h->geo.n, h->geo.n_det, af, asub, M, NP);
  if (!qs.ok || qs.pieces.empty()) return MCR_OK;  // this variant is unavailable on this geometry
  // consecutive workgroups go to the 8 XCDs in turn: within each subset, sort
  // the pieces by the middle image row of their lines and cut them into 8
  // runs of equal line counts; run x goes to positions = x (mod 8), so that
  // each XCD's L2 holds about an eighth of the image planes; shorter runs are
  // padded with entries of unit -1
  std::vector<int4> ordered;
  std::vector<int2> sub_pieces(M);
  for (int sb = 0; sb < M; ++sb) {
    const int2 r = qs.sub_pieces[sb];
    std::vector<std::pair<int, int4>> keyed;
    long total = 0;
    for (int q = r.x; q < r.x + r.y; ++q) {
      const int4& pc = qs.pieces[q];
      int lo = INT_MAX, hi = -1, lines = 0;
      for (int b = pc.x; b < pc.x + pc.y; ++b) {
        lo = std::min(lo, qs.bands[b].x);
        hi = std::max(hi, qs.bands[b].x + qs.bands[b].y - 1);
        lines += qs.bands[b].y;
      }
      keyed.push_back({hi >= lo ? (lo + hi) / 2 : 0, pc});
      total += lines;
    }
    std::stable_sort(keyed.begin(), keyed.end(),
                     [](const std::pair<int, int4>& a, const std::pair<int, int4>& b) { return a.first < b.first; });
    std::vector<std::vector<int4>> bucket(8);
    long cum = 0;
    for (const auto& kp : keyed) {
      const int4& pc = kp.second;
      bucket[std::min<long>(7, total > 0 ? 8 * cum / total : 0)].push_back(pc);
      for (int b = pc.x; b < pc.x + pc.y; ++b) cum += qs.bands[b].y;
    }
    size_t len = 0;
    for (const auto& bk : bucket) len = std::max(len, bk.size());
    std::vector<int4> order(8 * len, make_int4(0, 0, -1, 0));
    for (int x = 0; x < 8; ++x)
      for (size_t q = 0; q < bucket[x].size(); ++q) order[8 * q + x] = bucket[x][q];
    sub_pieces[sb] = make_int2((int)ordered.size(), (int)order.size());
    ordered.insert(ordered.end(), order.begin(), order.end());
  }
  qs.pieces = ordered;
  const int ns = h->nslots;
  if (!h->wf.wQ) STATUS_OK(dmalloc(h, (void**)&h->wf.wQ, sizeof(float) * 7 * h->padded * ns));
  qt.part_floats = qs.part_floats;
  STATUS_OK(dmalloc(h, (void**)&qt.chunks, sizeof(int4) * qs.chunks.size()));
  STATUS_OK(dmalloc(h, (void**)&qt.pieces, sizeof(int4) * qs.pieces.size()));
  STATUS_OK(dmalloc(h, (void**)&qt.units, sizeof(int4) * qs.units.size()));
  STATUS_OK(dmalloc(h, (void**)&qt.bands, sizeof(int4) * std::max<size_t>(1, qs.bands.size())));
  STATUS_OK(dmalloc(h, (void**)&qt.part, sizeof(float) * std::max<long>(1, qs.part_floats) * ns));
  STATUS_OK(dmalloc(h, (void**)&qt.multi, sizeof(int) * std::max<size_t>(1, qs.multi.size())));
  HIP_OK(hipMemcpyAsync(qt.chunks, qs.chunks.data(), sizeof(int4) * qs.chunks.size(), hipMemcpyHostToDevice,
                        h->stream));
  HIP_OK(hipMemcpyAsync(qt.pieces, qs.pieces.data(), sizeof(int4) * qs.pieces.size(), hipMemcpyHostToDevice,
                        h->stream));
  HIP_OK(hipMemcpyAsync(qt.units, qs.units.data(), sizeof(int4) * qs.units.size(), hipMemcpyHostToDevice,
                        h->stream));
  if (!qs.bands.empty())
    HIP_OK(hipMemcpyAsync(qt.bands, qs.bands.data(), sizeof(int4) * qs.bands.size(), hipMemcpyHostToDevice,
                          h->stream));
  if (!qs.multi.empty())
    HIP_OK(hipMemcpyAsync(qt.multi, qs.multi.data(), sizeof(int) * qs.multi.size(), hipMemcpyHostToDevice,
                          h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  qt.npieces = (int)qs.pieces.size();
  qt.nmulti = (int)qs.multi.size();
  if (by_subset) {
    qt.sub = sub_pieces;
    qt.sub_multi = qs.sub_multi;
  }
  return MCR_OK;
}

mcr_status upload_quad(mcr_handle* h, const std::vector<AngleFx>& af) {
  HIP_OK(hipStreamSynchronize(h->stream));
  STATUS_OK(upload_quad_tables(h, af, 0));
  return upload_quad_tables(h, af, 1);
}

// Quarter-turn adjoint codes (adj_px < 0): -2, -4, -8 = 2, 4, 8 pixels per
// thread on 32 x 8PX tiles (256 threads), -16 = 4 pixels on 32 x 64 tiles
// (512 threads), -32 = 4 pixels on 64 x 64 tiles (1024 threads). Where the
// geometry has no quarter-turn symmetry the tiled kernel runs with the
// pixels per thread returned here.
int quad_tiled_px(int code) { return code >= -8 ? -code : 8; }

// The quarter-turn adjoint pairs angle k with angle k +- n_angles/2 and a
// pixel with its quarter turns: it needs an even image size, an even number
// of angles, and all of them in the launch (all angles, or a subset whose
// angles come with their partners k +- n_a/2: the paired partition). Its
// sinogram loads take 32-bit byte offsets within one slot: 4 n_a n_d < 2^31.
bool quad_ok(const mcr_handle* h, const AngleRanges& ar) {
  const int na = h->geo.n_angles;
  const bool all = ar.ka == 0 && ar.kb == na && ar.kd == ar.kc;
  const bool paired = ar.kc == ar.ka + na / 2 && ar.kd == ar.kb + na / 2;
  const bool fits = 4L * na * h->geo.n_det < (1L << 31);
  return h->geo.n % 2 == 0 && na % 2 == 0 && fits && (all || paired);
}

AngleRanges subset_ranges(const mcr_handle* h, int subset) {
  if (subset < 0 || h->M == 1) return AngleRanges{0, h->geo.n_angles, 0, 0};
  return h->sub[subset];
}

template <typename T>
mcr_status init_work(mcr_handle* h) {
  Work<T>& w = work<T>(h);
  if (w.ready) return MCR_OK;
  const int N = h->N;
  const long n2 = (long)h->geo.n * h->geo.n;
  STATUS_OK(dmalloc(h, (void**)&w.ang, sizeof(AngleT<T>) * h->geo.n_angles));
  STATUS_OK(dmalloc(h, (void**)&w.motion, sizeof(GateMotion<T>) * (N + 1)));
  w.sc_cap = N * h->M;
  STATUS_OK(dmalloc(h, (void**)&w.scalars, sizeof(GateScalars<T>) * w.sc_cap));
  STATUS_OK(dmalloc(h, (void**)&w.ptrs, sizeof(GatePtrs<T>) * N));
  const int ns = h->nslots;
  STATUS_OK(dmalloc(h, (void**)&w.wP, sizeof(T) * h->padded * ns));
  STATUS_OK(dmalloc(h, (void**)&w.wTP, sizeof(T) * h->padded * ns));
  STATUS_OK(dmalloc(h, (void**)&w.bP, sizeof(T) * h->padded * ns));
  STATUS_OK(dmalloc(h, (void**)&w.dy, sizeof(T) * h->sino * ns));
  STATUS_OK(dmalloc(h, (void**)&w.img, sizeof(T) * n2));
  STATUS_OK(dmalloc(h, (void**)&w.img2, sizeof(T) * n2));
  w.pin_bytes = sizeof(GateScalars<T>) * w.sc_cap + sizeof(GatePtrs<T>) * N;
  HIP_OK(hipHostMalloc(&w.pin, w.pin_bytes, hipHostMallocDefault));
  HIP_OK(hipEventCreateWithFlags(&w.pin_ev, hipEventDisableTiming));
  const std::vector<AngleT<T>> at = angle_table<T>(h->geo.n_angles);
  HIP_OK(hipMemcpyAsync(w.ang, at.data(), sizeof(AngleT<T>) * at.size(), hipMemcpyHostToDevice, h->stream));
  STATUS_OK(dmalloc(h, (void**)&w.angfx, sizeof(AngleFx) * h->geo.n_angles));
  const std::vector<AngleFx> af = angle_table_fx(h->geo.n, h->geo.n_angles, h->geo.n_det);
  HIP_OK(hipMemcpyAsync(w.angfx, af.data(), sizeof(AngleFx) * af.size(), hipMemcpyHostToDevice, h->stream));
  if constexpr (std::is_same<T, float>::value) {
    std::vector<int2> ch = angle_chunks(af, kFwdKA);
    h->fwd_lds_ok = tiled_windows_fit(h, af, ch);
    h->nchunks = (int)ch.size();
    STATUS_OK(dmalloc(h, (void**)&h->chunks, sizeof(int2) * ch.size()));
    HIP_OK(hipMemcpyAsync(h->chunks, ch.data(), sizeof(int2) * ch.size(), hipMemcpyHostToDevice, h->stream));
    STATUS_OK(dmalloc(h, (void**)&h->parts, sizeof(float) * kMaxShares * ns * n2));
    const Schedule sc = build_schedule(h->geo.n, h->geo.n_det, af, kFwdKA, kFwdJD, kFwdWL);
    h->sched_ok = sc.ok;
    h->sched_nchunks = (int)sc.chunks.size();
    STATUS_OK(dmalloc(h, (void**)&h->sched_chunks, sizeof(int4) * sc.chunks.size()));
    STATUS_OK(dmalloc(h, (void**)&h->sched_blocks, sizeof(int2) * sc.blocks.size()));
    STATUS_OK(dmalloc(h, (void**)&h->sched_bands, sizeof(int4) * std::max<size_t>(1, sc.bands.size())));
    HIP_OK(hipMemcpyAsync(h->sched_chunks, sc.chunks.data(), sizeof(int4) * sc.chunks.size(), hipMemcpyHostToDevice,
                          h->stream));
    HIP_OK(hipMemcpyAsync(h->sched_blocks, sc.blocks.data(), sizeof(int2) * sc.blocks.size(), hipMemcpyHostToDevice,
                          h->stream));
    if (!sc.bands.empty())
      HIP_OK(hipMemcpyAsync(h->sched_bands, sc.bands.data(), sizeof(int4) * sc.bands.size(), hipMemcpyHostToDevice,
                            h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    STATUS_OK(upload_shear(h, af));
    STATUS_OK(upload_quad(h, af));
  }
  HIP_OK(hipStreamSynchronize(h->stream));
  STATUS_OK(upload_motion<T>(h));
  w.ready = true;
  return MCR_OK;
}

// Uploads per-gate scalars and pointers when they differ from the last upload.
// The pinned buffer is only rewritten after the previous copy has executed.
template <typename T>
mcr_status upload_params(mcr_handle* h, const std::vector<GateScalars<T>>& sc,
                         const std::vector<GatePtrs<T>>& pt) {
  Work<T>& w = work<T>(h);
  const size_t b1 = sizeof(GateScalars<T>) * sc.size(), b2 = sizeof(GatePtrs<T>) * pt.size();
  std::vector<char> cur(b1 + b2);
  std::memcpy(cur.data(), sc.data(), b1);
  std::memcpy(cur.data() + b1, pt.data(), b2);
  if (cur == w.last) return MCR_OK;
  if (w.pin_recorded) HIP_OK(hipEventSynchronize(w.pin_ev));
  std::memcpy(w.pin, cur.data(), cur.size());
  HIP_OK(hipMemcpyAsync(w.scalars, w.pin, b1, hipMemcpyHostToDevice, h->stream));
  HIP_OK(hipMemcpyAsync(w.ptrs, (char*)w.pin + b1, b2, hipMemcpyHostToDevice, h->stream));
  HIP_OK(hipEventRecord(w.pin_ev, h->stream));
  w.pin_recorded = true;
  w.last.swap(cur);
  return MCR_OK;
}

int max_radius(const mcr_handle* h, int gate0, int G) {
  int r = 1;
  for (int i = gate0; i < gate0 + G && i < h->N; ++i) r = std::max(r, h->radius[i]);
  return r;
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
template <typename T>
mcr_status launch_warp(mcr_handle* h, int gate0, int G, const T* x, const SlotInfo* slots = nullptr,
                       long x_stride = 0) {
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  Timed tm(h, MCR_KERNEL_WARP);
  dim3 grid(cdiv(n, 32), cdiv(n, 32), G), block(32, 32);
  // the quarter-turn planes only when the forward that reads them is
  // selected (three, or seven with the transposes); the transposed image only
  // when some launch may use another forward (angle subsets of less than all
  // angles)
  const int fwd = h->tune.fwd;
  const bool quad = std::is_same<T, float>::value && ((fwd == 4 && h->qt[0].npieces > 0) ||
                                                      (fwd == 5 && h->qt[1].npieces > 0));
  const int nq = quad ? (fwd == 5 ? 7 : 3) : 0;
  const bool sub_quad = h->sub_paired && !h->qt[0].sub.empty();
  T* wQ = quad ? w.wQ : nullptr;
  T* wT = quad && (h->M == 1 || sub_quad) ? nullptr : w.wTP;
  hipLaunchKernelGGL(k_warp_fwd<T>, grid, block, 0, h->stream, geo_of<T>(h), w.motion, gate0,
                     h->fieldP, 2 * h->padded, h->padded, x, x_stride, w.wP, wT, h->padded, slots, wQ,
                     7 * h->padded, h->padded, nq);
  LAUNCH_OK();
  return MCR_OK;
}

// Angles of subset `subset` (-1: all angles).
AngleRanges subset_ranges(const mcr_handle* h, int subset);
bool quad_ok(const mcr_handle* h, const AngleRanges& ar);
int quad_tiled_px(int code);

template <typename T, int MODE>
mcr_status launch_project(mcr_handle* h, int gate0, int G, T* out, long out_stride,
                          const SlotInfo* slots = nullptr, int subset = -1) {
  Work<T>& w = work<T>(h);
  Timed tm(h, MCR_KERNEL_PROJECT);
  const AngleRanges ar = subset_ranges(h, subset);
  const GateScalars<T>* gs = w.scalars + w.sc_base;
  const dim3 block(256);
  if constexpr (std::is_same<T, float>::value) {
    // the chunk tables of variants 1 and 2 cover all angles; those of variant
    // 4 all angles or each paired subset, those of variant 5 all angles (a
    // subset launch of variant 5 runs variant 4, whose planes the warp also
    // wrote)
    const bool part = subset >= 0 && h->M > 1;
    const bool sub_quad = h->sub_paired && !h->qt[0].sub.empty();
    int fwd = h->tune.fwd;
    if (part && fwd == 5) fwd = 4;
    if (part && !(fwd == 0 || fwd == 3 || (fwd == 4 && sub_quad))) fwd = h->shear_npieces > 0 ? 3 : 0;
    if ((fwd == 4 && h->qt[0].npieces > 0) || (fwd == 5 && h->qt[1].npieces > 0)) {
      const QuadTables& qt = h->qt[fwd == 5];
      const int2 pr = part ? qt.sub[subset] : make_int2(0, qt.npieces);
      const int2 mr = part ? qt.sub_multi[subset] : make_int2(0, qt.nmulti);
#define FWDQ(NP)                                                                                                    \
  do {                                                                                                              \
    if (pr.y > 0) {                                                                                                 \
      hipLaunchKernelGGL((k_joseph_fwd_quad<MODE, NP>), dim3(pr.y, 1, G), dim3(256), 0, h->stream, geo_of<T>(h),   \
                         w.angfx, qt.chunks, qt.pieces, qt.units, qt.bands, w.wP, w.wQ, h->padded, 7 * h->padded,  \
                         h->padded, out, out_stride, gate0, gs, w.ptrs, slots, qt.part, qt.part_floats, pr.x);      \
      LAUNCH_OK();                                                                                                  \
    }                                                                                                               \
    if (mr.y > 0)                                                                                                   \
      hipLaunchKernelGGL((k_joseph_fwd_quad_finish<MODE, NP>), dim3(mr.y, NP, G), dim3(256), 0, h->stream,          \
                         geo_of<T>(h), w.angfx, qt.chunks, qt.units, qt.multi, qt.part, qt.part_floats, out,        \
                         out_stride, gate0, gs, w.ptrs, slots, mr.x);                                               \
  } while (0)
      if (fwd == 5)
        FWDQ(8);
      else
        FWDQ(4);
#undef FWDQ
    } else if (fwd == 3 && h->shear_npieces > 0) {
      const int2 pr = subset >= 0 ? h->shear_sub[subset] : make_int2(0, h->shear_npieces);
      const int2 mr = subset >= 0 ? h->shear_sub_multi[subset] : make_int2(0, h->shear_nmulti);
      if (pr.y > 0) {
        hipLaunchKernelGGL((k_joseph_fwd_shear<MODE>), dim3(pr.y, 1, G), dim3(256), 0, h->stream, geo_of<T>(h),
                           w.angfx, h->shear_chunks, h->shear_pieces, h->shear_units, h->shear_bands, w.wP, w.wTP,
                           h->padded, out, out_stride, gate0, gs, w.ptrs, slots, h->shear_part, h->shear_part_floats,
                           pr.x);
        LAUNCH_OK();
      }
      if (mr.y > 0) {
        hipLaunchKernelGGL((k_joseph_fwd_shear_finish<MODE>), dim3(mr.y, 1, G), dim3(256), 0, h->stream,
                           geo_of<T>(h), w.angfx, h->shear_chunks, h->shear_units, h->shear_multi, h->shear_part,
                           h->shear_part_floats, out, out_stride, gate0, gs, w.ptrs, slots, mr.x);
      }
    } else if (fwd == 2 && h->sched_ok) {
      dim3 gt(cdiv(h->geo.n_det, kFwdJD), h->sched_nchunks, G);
      hipLaunchKernelGGL((k_joseph_fwd_sched<kFwdKA, kFwdJD, kFwdWL, MODE>), gt, dim3(256), 0, h->stream,
                         geo_of<T>(h), w.angfx, h->sched_chunks, h->sched_blocks, h->sched_bands, w.wP, w.wTP,
                         h->padded, out, out_stride, gate0, gs, w.ptrs, slots);
    } else if (fwd == 1 && h->fwd_lds_ok) {
      dim3 gt(cdiv(h->geo.n_det, kFwdJD), h->nchunks, G);
      hipLaunchKernelGGL((k_joseph_fwd_lds<kFwdKA, kFwdJD, kFwdWL, MODE>), gt, dim3(256), 0, h->stream,
                         geo_of<T>(h), w.angfx, h->chunks, w.wP, w.wTP, h->padded, out, out_stride, gate0, gs,
                         w.ptrs, slots);
    } else {
      for (int part_r = 0; part_r < 2; ++part_r) {  // one launch per angle range
        const int k0 = part_r ? ar.kc : ar.ka, cnt = part_r ? ar.kd - ar.kc : ar.kb - ar.ka;
        if (cnt <= 0) continue;
        hipLaunchKernelGGL((k_joseph_fwd_fx<MODE>), dim3(cdiv(h->geo.n_det, 256), cnt, G), block, 0, h->stream,
                           geo_of<T>(h), w.angfx, w.wP, w.wTP, h->padded, out, out_stride, gate0, gs, w.ptrs, slots,
                           k0);
        LAUNCH_OK();
      }
    }
  } else {
    for (int part_r = 0; part_r < 2; ++part_r) {
      const int k0 = part_r ? ar.kc : ar.ka, cnt = part_r ? ar.kd - ar.kc : ar.kb - ar.ka;
      if (cnt <= 0) continue;
      hipLaunchKernelGGL((k_joseph_fwd<T, MODE>), dim3(cdiv(h->geo.n_det, 256), cnt, G), block, 0, h->stream,
                         geo_of<T>(h), w.ang, w.wP, w.wTP, h->padded, out, out_stride, gate0, gs, w.ptrs, slots, k0);
      LAUNCH_OK();
    }
  }
  LAUNCH_OK();
  return MCR_OK;
}

// Fixed-order sum of the S partial backprojections of G slots; four pixels
// per thread where rows and the output are 16-byte aligned.
void launch_sum_parts(mcr_handle* h, int G, int S, long part_stride, float* out, long out_stride, int padded) {
  const int n = h->geo.n;
  const long n2 = (long)n * n;
  if (n % 4 == 0 && (uintptr_t)out % 16 == 0 && out_stride % 4 == 0)
    hipLaunchKernelGGL(k_sum_parts4, dim3(cdiv(n, 64), cdiv(n, 16), G), dim3(16, 16), 0, h->stream, n, h->pitch, S,
                       h->parts, part_stride, n2, out, out_stride, padded);
  else
    hipLaunchKernelGGL(k_sum_parts, dim3(cdiv(n, 16), cdiv(n, 16), G), dim3(16, 16), 0, h->stream, n, h->pitch, S,
                       h->parts, part_stride, n2, out, out_stride, padded);
}

template <typename T>
mcr_status launch_backproject(mcr_handle* h, int G, const T* sino, long sino_stride, T* out,
                              long out_stride, int padded, int subset = -1) {
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  Timed tm(h, MCR_KERNEL_BACKPROJECT);
  const AngleRanges ar = subset_ranges(h, subset);
  dim3 grid(cdiv(n, 16), cdiv(n, 16), G), block(16, 16);
  if constexpr (std::is_same<T, float>::value) {
    // adj_px < 0: the quarter-turn kernel where the geometry allows it (even
    // n and n_angles, all angles or a paired subset), else the tiled kernel
    // (quad_tiled_px)
    const int code = h->tune.adj_px;
    const bool quad = code < 0 && quad_ok(h, ar);
    const int px = code < 0 ? quad_tiled_px(code) : code, S = px > 0 ? h->tune.adj_s : 1;
    if (quad) {
      const long n2 = (long)n * n;
      float* dst = S > 1 ? h->parts : out;
      const long dst_stride = S > 1 ? n2 : out_stride;
      const long part_stride = n2 * h->nslots;
#define ADJQ(PX, TX, TY)                                                                                          \
  hipLaunchKernelGGL((k_joseph_adj_quad<PX, TX, TY>), dim3(cdiv(n / 2, TX * PX), cdiv(n / 2, TY), G * S),         \
                     dim3(TX * TY), 0, h->stream, geo_of<T>(h), w.angfx, sino, sino_stride, dst, dst_stride, padded, \
                     S, part_stride, ar)
      if (code == -2)
        ADJQ(2, 8, 32);
      else if (code == -4)
        ADJQ(4, 8, 32);
      else if (code == -8)
        ADJQ(8, 8, 32);
      else if (code == -16)
        ADJQ(4, 16, 32);
      else
        ADJQ(4, 16, 64);
#undef ADJQ
      LAUNCH_OK();
      if (S > 1) {
        launch_sum_parts(h, G, S, part_stride, out, out_stride, padded);
      }
    } else if (px > 0) {
      const long n2 = (long)n * n;
      // S > 1: partial images per angle share, then a fixed-order sum
      float* dst = S > 1 ? h->parts : out;
      const long dst_stride = S > 1 ? n2 : out_stride;
      const long part_stride = n2 * h->nslots;
      dim3 gt(cdiv(n, 8 * px), cdiv(n, 32), G * S);
#define ADJ(PX)                                                                                           \
  hipLaunchKernelGGL(k_joseph_adj_lds<PX>, gt, dim3(256), 0, h->stream, geo_of<T>(h), w.angfx, sino, \
                     sino_stride, dst, dst_stride, padded, S, part_stride, ar)
      if (px == 1)
        ADJ(1);
      else if (px == 2)
        ADJ(2);
      else if (px == 4)
        ADJ(4);
      else
        ADJ(8);
#undef ADJ
      LAUNCH_OK();
      if (S > 1) {
        launch_sum_parts(h, G, S, part_stride, out, out_stride, padded);
      }
    } else {
      hipLaunchKernelGGL(k_joseph_adj_fx, grid, block, 0, h->stream, geo_of<T>(h), w.angfx, sino,
                         sino_stride, out, out_stride, padded, ar);
    }
  } else
    hipLaunchKernelGGL(k_joseph_adj<T>, grid, block, 0, h->stream, geo_of<T>(h), w.ang, sino,
                       sino_stride, out, out_stride, padded, ar);
  LAUNCH_OK();
  return MCR_OK;
}

template <typename T, int MODE>
mcr_status launch_twarp(mcr_handle* h, int gate0, int G, T* out, UpdateArgs<T> ua, const SlotInfo* slots = nullptr,
                        int nslots = 0, const T* slice_tc = nullptr, int radius = 0) {
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  Timed tm(h, MCR_KERNEL_TWARP);
  dim3 grid(cdiv(n, 32), cdiv(n, 8), slots ? nslots : 1), block(32, 8);
  const int R = slots ? radius : max_radius(h, gate0, G);
  const Geo<T> g = geo_of<T>(h);
#define TW(RR)                                                                                   \
  hipLaunchKernelGGL((k_twarp<T, MODE, RR>), grid, block, 0, h->stream, g, w.motion, gate0, G,   \
                     w.scalars + w.sc_base, h->fieldP, 2 * h->padded, h->padded, h->centres, w.bP, h->padded, \
                     out, ua, slots, (long)n * n, slice_tc)
  if (R <= 1)
    TW(1);
  else if (R == 2)
    TW(2);
  else
    TW(3);
#undef TW
  LAUNCH_OK();
  return MCR_OK;
}

template <typename T>
mcr_status launch_xstep(mcr_handle* h, T* x, const T* zbar, T tau, T cx) {
  const long n2 = (long)h->geo.n * h->geo.n;
  Timed tm(h, MCR_KERNEL_XSTEP);
  hipLaunchKernelGGL(k_xstep<T>, dim3(cdiv(n2, 256)), dim3(256), 0, h->stream, n2, x, zbar, tau, cx);
  LAUNCH_OK();
  return MCR_OK;
}

template <typename T>
__global__ void k_from_padded(int n, int pitch, const T* __restrict__ src, T* __restrict__ dst) {
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c < n && r < n) dst[(long)r * n + c] = src[(long)(r + kPad) * pitch + c + kPad];
}

// Reductions into result slot `slot` of red_out (device); read back later.
template <typename Ta, typename Tb, int OP>
mcr_status launch_reduce(mcr_handle* h, long count, const Ta* a, const Tb* b, int slot) {
  Timed tm(h, MCR_KERNEL_OTHER);
  hipLaunchKernelGGL((k_reduce_partial<Ta, Tb, OP>), dim3(kRedBlocks), dim3(256), 0, h->stream, count,
                     a, b, h->red_partial);
  LAUNCH_OK();
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, h->stream, h->red_partial, h->red_out, slot);
  LAUNCH_OK();
  return MCR_OK;
}

mcr_status read_results(mcr_handle* h, int count) {
  HIP_OK(hipMemcpyAsync(h->red_host, h->red_out, sizeof(double) * count, hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  return MCR_OK;
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
mcr_status check_handle(const mcr_handle* h) {
  if (!h) return fail(MCR_ERR_ARG, "null handle");
  return MCR_OK;
}

mcr_status check_gate(const mcr_handle* h, int gate) {
  if (gate < 0 || gate >= h->N) return fail(MCR_ERR_ARG, "gate %d out of range [0, %d)", gate, h->N);
  return MCR_OK;
}

mcr_status check_ptr(const void* p, const char* what) {
  if (!p) return fail(MCR_ERR_ARG, "%s is null", what);
  return MCR_OK;
}

mcr_status check_motion(const mcr_motion* m, int i) {
  if (m->kind < MCR_MOTION_IDENTITY || m->kind > MCR_MOTION_FIELD)
    return fail(MCR_ERR_ARG, "gate %d: unknown motion kind %d", i, m->kind);
  if (m->kind == MCR_MOTION_RIGID)
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(m->rigid[k])) return fail(MCR_ERR_ARG, "gate %d: rigid parameter %d not finite", i, k);
  if (m->kind == MCR_MOTION_FIELD && !m->field) return fail(MCR_ERR_ARG, "gate %d: field pointer is null", i);
  return MCR_OK;
}

mcr_status check_alg(const mcr_handle* h, const mcr_state* st, const void* const* d, double alpha,
                     const double* sigma, double tau, double theta, const double* p) {
  if (!st) return fail(MCR_ERR_ARG, "state is null");
  STATUS_OK(check_ptr(st->x, "state.x"));
  STATUS_OK(check_ptr(st->z, "state.z"));
  STATUS_OK(check_ptr(st->zbar, "state.zbar"));
  STATUS_OK(check_ptr(st->y, "state.y"));
  STATUS_OK(check_ptr(d, "d"));
  STATUS_OK(check_ptr(sigma, "sigma"));
  for (int i = 0; i < h->N; ++i) {
    if (!st->y[i]) return fail(MCR_ERR_ARG, "state.y[%d] is null", i);
    if (!d[i]) return fail(MCR_ERR_ARG, "d[%d] is null", i);
    if (!(sigma[i] > 0) || !std::isfinite(sigma[i]))
      return fail(MCR_ERR_ARG, "sigma[%d] = %g must be finite and > 0", i, sigma[i]);
    if (p && (!(p[i] > 0) || !(p[i] <= 1))) return fail(MCR_ERR_ARG, "p[%d] = %g must be in (0, 1]", i, p[i]);
  }
  if (!(alpha > 0) || !std::isfinite(alpha)) return fail(MCR_ERR_ARG, "alpha = %g must be finite and > 0", alpha);
  if (!(tau > 0) || !std::isfinite(tau)) return fail(MCR_ERR_ARG, "tau = %g must be finite and > 0", tau);
  if (!(theta >= 0) || !std::isfinite(theta)) return fail(MCR_ERR_ARG, "theta = %g must be finite and >= 0", theta);
  return MCR_OK;
}

// ---------------------------------------------------------------------------
// Algorithm 1 driver: one iteration over the gates gate0 .. gate0+G-1.
// ---------------------------------------------------------------------------
// subset >= 0: the block (gate, subset) of the gates x angle-subsets
// sampling; its scalars are entry subset * N + gate.
template <typename T>
mcr_status iteration(mcr_handle* h, const mcr_state* st, int gate0, int G, bool xstep_first,
                     bool xstep_after, T tau, T cx, int subset = -1) {
  Work<T>& w = work<T>(h);
  T* x = (T*)st->x;
  if (xstep_first) STATUS_OK(launch_xstep<T>(h, x, (const T*)st->zbar, tau, cx));
  w.sc_base = subset > 0 ? subset * h->N : 0;
  mcr_status rc = launch_warp<T>(h, gate0, G, x);
  if (rc == MCR_OK) rc = launch_project<T, 1>(h, gate0, G, w.dy, h->sino, nullptr, subset);
  if (rc == MCR_OK) rc = launch_backproject<T>(h, G, w.dy, h->sino, w.bP, h->padded, 1, subset);
  UpdateArgs<T> ua{x, (T*)st->z, (T*)st->zbar, tau, cx, xstep_after ? 1 : 0};
  if (rc == MCR_OK) rc = launch_twarp<T, 2>(h, gate0, G, nullptr, ua);
  w.sc_base = 0;
  return rc;
}

// Scalar tables for N M blocks (grown when the subset count grows).
template <typename T>
mcr_status ensure_scalars(mcr_handle* h) {
  Work<T>& w = work<T>(h);
  if (!w.ready || w.sc_cap >= h->N * h->M) return MCR_OK;
  HIP_OK(hipStreamSynchronize(h->stream));
  if (w.pin_recorded) HIP_OK(hipEventSynchronize(w.pin_ev));
  dfree(h, w.scalars);
  w.scalars = nullptr;
  w.sc_cap = h->N * h->M;
  STATUS_OK(dmalloc(h, (void**)&w.scalars, sizeof(GateScalars<T>) * w.sc_cap));
  HIP_OK(hipHostFree(w.pin));
  w.pin = nullptr;
  w.pin_bytes = sizeof(GateScalars<T>) * w.sc_cap + sizeof(GatePtrs<T>) * h->N;
  HIP_OK(hipHostMalloc(&w.pin, w.pin_bytes, hipHostMallocDefault));
  w.pin_recorded = false;
  w.last.clear();
  return MCR_OK;
}

// Block b = gate * M + subset has sigma[b], p[b]; its scalars go to entry
// subset * N + gate, where the launches of an iteration on that subset look.
template <typename T>
mcr_status set_params_blocks(mcr_handle* h, const mcr_state* st, const void* const* d, const double* sigma,
                             double theta, const double* p) {
  const int N = h->N, M = h->M;
  std::vector<GateScalars<T>> sc(N * M);
  std::vector<GatePtrs<T>> pt(N);
  for (int i = 0; i < N; ++i) {
    for (int s = 0; s < M; ++s) {
      const int b = i * M + s;
      GateScalars<T>& e = sc[s * N + i];
      e.sigma = T(sigma[b]);
      e.cy = T(1.0 / (1.0 + sigma[b] * N / 2.0));
      e.coef = T(theta / p[b]);
      e.pad_ = T(0);
    }
    pt[i].y = (T*)st->y[i];
    pt[i].d = (const T*)d[i];
  }
  Work<T>& w = work<T>(h);
  w.sc_host = sc;
  w.pt_host = pt;
  return upload_params<T>(h, sc, pt);
}

template <typename T>
mcr_status spdhg_blocks_impl(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha,
                             const double* sigma, double tau, double theta, const double* p, const int32_t* seq,
                             int n_iter) {
  STATUS_OK(set_params_blocks<T>(h, st, d, sigma, theta, p));
  const T t = T(tau), cx = T(1.0 / (1.0 + 2.0 * tau * alpha));
  for (int k = 0; k < n_iter; ++k)
    STATUS_OK(iteration<T>(h, st, seq[k] / h->M, 1, k == 0, k + 1 < n_iter, t, cx, seq[k] % h->M));
  return MCR_OK;
}

template <typename T>
mcr_status set_params(mcr_handle* h, const mcr_state* st, const void* const* d, const double* sigma,
                      double theta, const double* p) {
  const int N = h->N;
  std::vector<GateScalars<T>> sc(N);
  std::vector<GatePtrs<T>> pt(N);
  for (int i = 0; i < N; ++i) {
    sc[i].sigma = T(sigma[i]);
    sc[i].cy = T(1.0 / (1.0 + sigma[i] * N / 2.0));
    sc[i].coef = T(theta / (p ? p[i] : 1.0));
    sc[i].pad_ = T(0);
    pt[i].y = (T*)st->y[i];
    pt[i].d = (const T*)d[i];
  }
  Work<T>& w = work<T>(h);
  w.sc_host = sc;
  w.pt_host = pt;
  return upload_params<T>(h, sc, pt);
}

// ---------------------------------------------------------------------------
// Differentiation through unrolled SPDHG iterations
// ---------------------------------------------------------------------------
template <typename T>
mcr_status launch_motion_grad(mcr_handle* h, int gate, const T* hP, const T* v, void* gmot) {
  const int kind = h->motion[gate].kind;
  if (kind == MCR_MOTION_IDENTITY || !gmot) return MCR_OK;
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  Timed tm(h, MCR_KERNEL_OTHER);
  dim3 grid(cdiv(n, 16), cdiv(n, 16)), block(16, 16);
  hipLaunchKernelGGL(k_motion_grad<T>, grid, block, 0, h->stream, geo_of<T>(h), w.motion, gate, h->fieldP,
                     2 * h->padded, h->padded, hP, v, h->mgrad_partial, (T*)gmot);
  LAUNCH_OK();
  if (kind == MCR_MOTION_RIGID) {
    hipLaunchKernelGGL(k_motion_grad_final, dim3(1), dim3(256), 0, h->stream, h->mgrad_partial,
                       (int)(grid.x * grid.y), (double*)gmot);
    LAUNCH_OK();
  }
  return MCR_OK;
}

template <typename T>
mcr_status spdhg_ckpt_impl(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha,
                           const double* sigma, double tau, double theta, const double* p, const int32_t* seq,
                           int n_iter, void* const* x1c, void* const* yc, void* const* bc) {
  STATUS_OK(set_params<T>(h, st, d, sigma, theta, p));
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  const T t = T(tau), cx = T(1.0 / (1.0 + 2.0 * tau * alpha));
  const long n2 = (long)h->geo.n * h->geo.n;
  for (int k = 0; k < n_iter; ++k) {
    const int g = seq[k];
    STATUS_OK(launch_xstep<T>(h, (T*)st->x, (const T*)st->zbar, t, cx));
    HIP_OK(hipMemcpyAsync(x1c[k], st->x, sizeof(T) * n2, hipMemcpyDeviceToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(yc[k], st->y[g], sizeof(T) * h->sino, hipMemcpyDeviceToDevice, h->stream));
    STATUS_OK(iteration<T>(h, st, g, 1, false, false, t, cx));
    if (bc) {  // the iteration's backprojection, still in the padded work image
      hipLaunchKernelGGL(k_from_padded<T>, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0, h->stream, n, h->pitch,
                         w.bP, (T*)bc[k]);
      LAUNCH_OK();
    }
  }
  return MCR_OK;
}

template <typename T>
mcr_status step_backward_impl(mcr_handle* h, int gate, const void* x1, const void* yb, const void* dg,
                              double alpha, double sigma, double tau, double theta, double p, void* gx,
                              void* gy, void* gz, void* gzb, void* gmot, const void* bck) {
  Work<T>& w = work<T>(h);
  const int N = h->N;
  const double cyd = 1.0 / (1.0 + sigma * N / 2.0);
  const long n2 = (long)h->geo.n * h->geo.n;
  const T cx = T(1.0 / (1.0 + 2.0 * tau * alpha));
  const dim3 gi(cdiv(n2, 256)), gs(cdiv(h->sino, 256)), blk(256);
  // b = A^T dy, dy = y1 - y: stored by the forward, or recomputed from the
  // checkpoint (the same kernels on the same inputs: the same values)
  if (bck) {
    const int n = h->geo.n;
    hipLaunchKernelGGL((k_to_padded<T, T>), dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0, h->stream, n, h->pitch,
                       (const T*)bck, w.bP);
    LAUNCH_OK();
  } else {
    // the recomputation's dual step reads the gate's scalars and pointers
    // from the device tables (their upload waits for the previous one)
    if ((int)w.sc_host.size() != N) {
      w.sc_host.assign(N, GateScalars<T>{});
      w.pt_host.assign(N, GatePtrs<T>{});
    }
    w.sc_host[gate] = GateScalars<T>{T(sigma), T(cyd), T(theta / p), T(0)};
    w.pt_host[gate] = GatePtrs<T>{(T*)yb, (const T*)dg};
    STATUS_OK(upload_params<T>(h, w.sc_host, w.pt_host));
    STATUS_OK(launch_warp<T>(h, gate, 1, (const T*)x1));
    STATUS_OK((launch_project<T, 2>(h, gate, 1, w.dy, h->sino)));
    STATUS_OK(launch_backproject<T>(h, 1, w.dy, h->sino, w.bP, h->padded, 1));
  }
  // z / z-bar
  {
    Timed tm(h, MCR_KERNEL_OTHER);
    hipLaunchKernelGGL(k_bwd_z<T>, gi, blk, 0, h->stream, n2, (T*)gz, (const T*)gzb, w.img, T(1.0 + theta / p));
    LAUNCH_OK();
  }
  // dz = D^T b: gb = D gdz, and the motion through D^T
  STATUS_OK(launch_motion_grad<T>(h, gate, w.bP, w.img, gmot));
  STATUS_OK(launch_warp<T>(h, gate, 1, w.img));
  // b = A^T dy, dy = y1 - y, y1 = c_y (y + sigma (s - d))
  STATUS_OK((launch_project<T, 0>(h, gate, 1, w.dy, h->sino)));
  {
    Timed tm(h, MCR_KERNEL_OTHER);
    hipLaunchKernelGGL(k_bwd_dual<T>, gs, blk, 0, h->stream, h->sino, (T*)gy, w.dy, T(cyd), T(sigma));
    LAUNCH_OK();
  }
  // s = A D x1: gw = A^T gs, gx1 = gx + D^T gw, and the motion through D
  STATUS_OK(launch_backproject<T>(h, 1, w.dy, h->sino, w.bP, h->padded, 1));
  STATUS_OK(launch_motion_grad<T>(h, gate, w.bP, (const T*)x1, gmot));
  STATUS_OK((launch_twarp<T, 1>(h, gate, 1, (T*)gx, UpdateArgs<T>{})));
  // x1 = c_x (x - tau zbar)
  {
    Timed tm(h, MCR_KERNEL_OTHER);
    hipLaunchKernelGGL(k_bwd_x<T>, gi, blk, 0, h->stream, n2, (T*)gx, (T*)gzb, cx, T(tau));
    LAUNCH_OK();
  }
  return MCR_OK;
}

template <typename T>
mcr_status motion_grad_impl(mcr_handle* h, int gate, const void* himg, const void* v, void* gmot) {
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  hipLaunchKernelGGL((k_to_padded<T, T>), dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0, h->stream, n,
                     h->pitch, (const T*)himg, w.bP);
  LAUNCH_OK();
  return launch_motion_grad<T>(h, gate, w.bP, (const T*)v, gmot);
}

template <typename T>
mcr_status spdhg_impl(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha,
                      const double* sigma, double tau, double theta, const double* p,
                      const int32_t* seq, int n_iter) {
  STATUS_OK(set_params<T>(h, st, d, sigma, theta, p));
  const T t = T(tau), cx = T(1.0 / (1.0 + 2.0 * tau * alpha));
  for (int k = 0; k < n_iter; ++k)
    STATUS_OK(iteration<T>(h, st, seq[k], 1, k == 0, k + 1 < n_iter, t, cx));
  return MCR_OK;
}

template <typename T>
mcr_status pdhg_impl(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha,
                     const double* sigma, double tau, double theta) {
  STATUS_OK(set_params<T>(h, st, d, sigma, theta, nullptr));
  const T t = T(tau), cx = T(1.0 / (1.0 + 2.0 * tau * alpha));
  return iteration<T>(h, st, 0, h->N, true, false, t, cx);
}

// Gradient descent on the scaled coordinates s of a registration (D of them)
// with Barzilai-Borwein step lengths (the first trial moves 1 px) and Armijo
// backtracking (sufficient decrease 1e-4, at most 40 halvings); stops after
// the first accepted step shorter than tol, at a zero gradient or after
// max_iter steps. eval(s, E, g) gives the energy and its gradient in s.
template <int D, typename Eval>
mcr_status minimise_bb(Eval eval, double* s, int max_iter, double tol, double& E, int& k) {
  auto dot = [](const double* a, const double* b) {
    double v = 0.0;
    for (int m = 0; m < D; ++m) v += a[m] * b[m];
    return v;
  };
  double g[D];
  STATUS_OK(eval(s, E, g));
  if (!std::isfinite(E)) return fail(MCR_ERR_NONFINITE, "registration energy is not finite (check ref and target)");
  double gn = std::sqrt(dot(g, g));
  double alpha = gn > 0 ? 1.0 / gn : 1.0;
  k = 0;
  while (k < max_iter && gn > 0) {
    double sn[D], gnew[D], En = 0.0;
    for (int t = 0; t < 41; ++t) {
      for (int m = 0; m < D; ++m) sn[m] = s[m] - alpha * g[m];
      STATUS_OK(eval(sn, En, gnew));
      if (En <= E - 1e-4 * alpha * gn * gn) break;
      alpha *= 0.5;
    }
    ++k;
    const double step = alpha * gn;
    double ds[D], dg[D];
    for (int m = 0; m < D; ++m) {
      ds[m] = sn[m] - s[m];
      dg[m] = gnew[m] - g[m];
      s[m] = sn[m];
      g[m] = gnew[m];
    }
    E = En;
    gn = std::sqrt(dot(g, g));
    if (step < tol) break;
    const double sy = dot(ds, dg);
    alpha = sy > 0 ? dot(ds, ds) / sy : 2.0 * alpha;
  }
  return MCR_OK;
}

// Rigid registration of a gate's image to the reference: E(theta) =
// |D(theta) ref - target|^2 / 2 over s = (phi (n - 1) / 2, t_x, t_y) (see
// mcr_register_rigid). Each evaluation: the warp, the residual, its squared
// norm (FP64 reduction) and J^T r (motion gradient).
template <typename T>
mcr_status register_rigid_impl(mcr_handle* h, int gate, const void* ref, const void* target, double* params,
                               int max_iter, double tol, double* loss, int32_t* steps) {
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  const double scale[3] = {(n - 1) / 2.0, 1.0, 1.0};
  double* gdev = h->red_out + 1;  // result slots 1..3
  auto eval = [&](const double* s, double& E, double* g) -> mcr_status {
    for (int m = 0; m < 3; ++m) h->motion[gate].rigid[m] = s[m] / scale[m];
    STATUS_OK(upload_motion<T>(h));
    STATUS_OK(launch_warp<T>(h, gate, 1, (const T*)ref));
    hipLaunchKernelGGL(k_residual_padded<T>, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0, h->stream, n,
                       h->pitch, w.wP, (const T*)target, w.bP);
    LAUNCH_OK();
    STATUS_OK((launch_reduce<T, T, 0>(h, h->padded, w.bP, w.bP, 0)));
    HIP_OK(hipMemsetAsync(gdev, 0, 3 * sizeof(double), h->stream));
    STATUS_OK(launch_motion_grad<T>(h, gate, w.bP, (const T*)ref, gdev));
    STATUS_OK(read_results(h, 4));
    E = 0.5 * h->red_host[0];
    for (int m = 0; m < 3; ++m) g[m] = h->red_host[1 + m] / scale[m];
    return MCR_OK;
  };
  double s[3], E = 0.0;
  int k = 0;
  for (int m = 0; m < 3; ++m) s[m] = params[m] * scale[m];
  STATUS_OK(minimise_bb<3>(eval, s, max_iter, tol, E, k));
  for (int m = 0; m < 3; ++m) params[m] = h->motion[gate].rigid[m] = s[m] / scale[m];
  STATUS_OK(upload_motion<T>(h));
  if (loss) *loss = E;
  if (steps) *steps = k;
  return MCR_OK;
}

// Affine registration of a field gate: u(p) = A (p - c) + t, theta = (A00,
// A01, A10, A11, t_x, t_y), over s = (A (n - 1) / 2, t) (see
// mcr_register_affine). Each evaluation writes the field into the gate's
// padded planes, warps, takes the residual and its squared norm, the field
// gradient planes (motion gradient) and their six moments.
template <typename T>
mcr_status register_affine_impl(mcr_handle* h, int gate, const void* ref, const void* target, double* params,
                                int max_iter, double tol, double* loss, int32_t* steps) {
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  const long n2 = (long)n * n;
  if (!h->reg_g) {
    STATUS_OK(dmalloc(h, &h->reg_g, sizeof(double) * 2 * n2));
    STATUS_OK(dmalloc(h, (void**)&h->reg_partial, sizeof(double) * 6 * kRedBlocks));
    STATUS_OK(dmalloc(h, (void**)&h->reg_field, sizeof(float) * 2 * n2));
  }
  const double rad = (n - 1) / 2.0;
  const double scale[6] = {rad, rad, rad, rad, 1.0, 1.0};
  float* fP = h->fieldP + (long)gate * 2 * h->padded;
  const dim3 grid(cdiv(n, 16), cdiv(n, 16)), block(16, 16);
  auto set_field = [&](const double* th) -> mcr_status {
    hipLaunchKernelGGL(k_affine_field, grid, block, 0, h->stream, n, h->pitch, h->padded, th[0], th[1], th[2], th[3],
                       th[4], th[5], fP);
    LAUNCH_OK();
    return MCR_OK;
  };
  auto eval = [&](const double* s, double& E, double* g) -> mcr_status {
    double th[6];
    for (int m = 0; m < 6; ++m) th[m] = s[m] / scale[m];
    STATUS_OK(set_field(th));
    STATUS_OK(launch_warp<T>(h, gate, 1, (const T*)ref));
    hipLaunchKernelGGL(k_residual_padded<T>, grid, block, 0, h->stream, n, h->pitch, w.wP, (const T*)target, w.bP);
    LAUNCH_OK();
    STATUS_OK((launch_reduce<T, T, 0>(h, h->padded, w.bP, w.bP, 0)));
    HIP_OK(hipMemsetAsync(h->reg_g, 0, sizeof(T) * 2 * n2, h->stream));
    STATUS_OK(launch_motion_grad<T>(h, gate, w.bP, (const T*)ref, h->reg_g));
    hipLaunchKernelGGL(k_affine_moments<T>, dim3(kRedBlocks), dim3(256), 0, h->stream, n, (const T*)h->reg_g,
                       h->reg_partial);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_affine_moments_final, dim3(1), dim3(256), 0, h->stream, h->reg_partial, h->red_out + 1);
    LAUNCH_OK();
    STATUS_OK(read_results(h, 7));
    E = 0.5 * h->red_host[0];
    for (int m = 0; m < 6; ++m) g[m] = h->red_host[1 + m] / scale[m];
    return MCR_OK;
  };
  double s[6], E = 0.0;
  int k = 0;
  for (int m = 0; m < 6; ++m) s[m] = params[m] * scale[m];
  STATUS_OK(minimise_bb<6>(eval, s, max_iter, tol, E, k));
  for (int m = 0; m < 6; ++m) params[m] = s[m] / scale[m];
  // install the result as the gate's field (gather-window set-up and check)
  STATUS_OK(set_field(params));
  for (int pl = 0; pl < 2; ++pl) {
    hipLaunchKernelGGL(k_from_padded<float>, grid, block, 0, h->stream, n, h->pitch, fP + pl * h->padded,
                       h->reg_field + pl * n2);
    LAUNCH_OK();
  }
  mcr_motion m{};
  m.kind = MCR_MOTION_FIELD;
  m.field = h->reg_field;
  STATUS_OK(mcr_set_motion(h, gate, &m));
  if (loss) *loss = E;
  if (steps) *steps = k;
  return MCR_OK;
}

// The gate's motion becomes the identity (its field planes may hold a map
// whose gather windows were never set up: a rejected or interrupted one).
mcr_status reset_gate_identity(mcr_handle* h, int gate) {
  h->motion[gate].kind = MCR_MOTION_IDENTITY;
  h->motion[gate].field = nullptr;
  h->radius[gate] = 1;
  ++h->config_gen;
  STATUS_OK(upload_motion<double>(h));
  if (h->wf.ready) STATUS_OK(upload_motion<float>(h));
  return MCR_OK;
}

// Dense displacement-field registration of a field gate (see
// mcr_register_field): descent on u [2][n][n] with the steps of minimise_bb,
// the vectors on the device. Each evaluation (the gate's field planes hold
// float32(u)): the warp, the residual and its squared norm, the motion
// gradient planes, the regulariser's gradient and energy, |g|^2.
template <typename T>
mcr_status register_field_impl(mcr_handle* h, int gate, const void* ref0, const void* target0, float* field,
                               double lam, const double* sigmas, int n_levels, int max_iter, double tol,
                               double* loss, int32_t* steps) {
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  const long n2 = (long)n * n;
  if (!h->reg_g) {
    STATUS_OK(dmalloc(h, &h->reg_g, sizeof(double) * 2 * n2));
    STATUS_OK(dmalloc(h, (void**)&h->reg_partial, sizeof(double) * 6 * kRedBlocks));
    STATUS_OK(dmalloc(h, (void**)&h->reg_field, sizeof(float) * 2 * n2));
  }
  if (!h->reg_dense) STATUS_OK(dmalloc(h, (void**)&h->reg_dense, sizeof(double) * 8 * n2));
  if (n_levels > 0 && !h->reg_blur) {
    STATUS_OK(dmalloc(h, (void**)&h->reg_blur, sizeof(double) * 3 * n2));
    STATUS_OK(dmalloc(h, (void**)&h->reg_w, sizeof(double) * (2 * kMaxBlurRadius + 1)));
  }
  const void* ref = ref0;
  const void* target = target0;
  double* u = h->reg_dense;
  double* g = u + 2 * n2;
  double* u1 = g + 2 * n2;
  double* g1 = u1 + 2 * n2;
  float* fP = h->fieldP + (long)gate * 2 * h->padded;
  const dim3 grid(cdiv(n, 16), cdiv(n, 16)), block(16, 16);
  auto eval = [&](double* gout, double& E, double& gsq) -> mcr_status {
    STATUS_OK(launch_warp<T>(h, gate, 1, (const T*)ref));
    hipLaunchKernelGGL(k_residual_padded<T>, grid, block, 0, h->stream, n, h->pitch, w.wP, (const T*)target, w.bP);
    LAUNCH_OK();
    STATUS_OK((launch_reduce<T, T, 0>(h, h->padded, w.bP, w.bP, 0)));
    HIP_OK(hipMemsetAsync(h->reg_g, 0, sizeof(T) * 2 * n2, h->stream));
    STATUS_OK(launch_motion_grad<T>(h, gate, w.bP, (const T*)ref, h->reg_g));
    hipLaunchKernelGGL(k_field_reg_grad<T>, dim3(kRedBlocks), dim3(256), 0, h->stream, n, h->pitch, h->padded, fP,
                       (const T*)h->reg_g, lam, gout, h->red_partial);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, h->stream, h->red_partial, h->red_out, 1);
    LAUNCH_OK();
    STATUS_OK((launch_reduce<double, double, 0>(h, 2 * n2, gout, gout, 2)));
    STATUS_OK(read_results(h, 3));
    E = 0.5 * h->red_host[0] + 0.5 * lam * h->red_host[1];
    gsq = h->red_host[2];
    return MCR_OK;
  };
  hipLaunchKernelGGL(k_field_load, grid, block, 0, h->stream, n, h->pitch, h->padded, (const float*)field, u, fP);
  LAUNCH_OK();
  // scale-space levels (none given: one level on the images themselves)
  double E = 0.0;
  int k_total = 0;
  std::vector<double> wts;
  for (int level = 0; level < std::max(1, n_levels); ++level) {
    const double sigma = n_levels > 0 ? sigmas[level] : 0.0;
    if (sigma > 0) {
      const int R = (int)(3.0 * sigma + 0.5);
      wts.assign(2 * R + 1, 0.0);
      double sum = 0.0;
      for (int j = -R; j <= R; ++j) sum += (wts[j + R] = std::exp(-double(j) * j / (2.0 * sigma * sigma)));
      for (double& v : wts) v /= sum;
      HIP_OK(hipMemcpyAsync(h->reg_w, wts.data(), sizeof(double) * wts.size(), hipMemcpyHostToDevice, h->stream));
      T* rb = (T*)h->reg_blur;
      T* tb = rb + n2;
      T* tmp = tb + n2;
      for (int im = 0; im < 2; ++im) {
        hipLaunchKernelGGL((k_blur<T, 1>), grid, block, 0, h->stream, n, R, h->reg_w,
                           (const T*)(im == 0 ? ref0 : target0), tmp);
        LAUNCH_OK();
        hipLaunchKernelGGL((k_blur<T, 0>), grid, block, 0, h->stream, n, R, h->reg_w, (const T*)tmp,
                           im == 0 ? rb : tb);
        LAUNCH_OK();
      }
      HIP_OK(hipStreamSynchronize(h->stream));  // the weights' host copy may go now
      ref = rb;
      target = tb;
    } else {
      ref = ref0;
      target = target0;
    }
    double gsq = 0.0;
    STATUS_OK(eval(g, E, gsq));
    if (!std::isfinite(E))
      return fail(MCR_ERR_NONFINITE, "registration energy is not finite (check ref, target and field)");
    double gn = std::sqrt(gsq);
    double alpha = gn > 0 ? 1.0 / gn : 1.0;
    int k = 0;
    while (k < max_iter && gn > 0) {
      double En = 0.0, gsqn = 0.0;
      for (int t = 0; t < 41; ++t) {
        hipLaunchKernelGGL(k_field_trial, grid, block, 0, h->stream, n, h->pitch, h->padded, u, g, alpha, u1, fP);
        LAUNCH_OK();
        STATUS_OK(eval(g1, En, gsqn));
        if (En <= E - 1e-4 * alpha * gn * gn) break;
        alpha *= 0.5;
      }
      ++k;
      const double step = alpha * gn;
      hipLaunchKernelGGL(k_dot_diff, dim3(kRedBlocks), dim3(256), 0, h->stream, 2 * n2, u1, u, g1, g, h->red_partial);
      LAUNCH_OK();
      hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, h->stream, h->red_partial, h->red_out, 0);
      LAUNCH_OK();
      hipLaunchKernelGGL(k_dot_diff, dim3(kRedBlocks), dim3(256), 0, h->stream, 2 * n2, u1, u, u1, u, h->red_partial);
      LAUNCH_OK();
      hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, h->stream, h->red_partial, h->red_out, 1);
      LAUNCH_OK();
      STATUS_OK(read_results(h, 2));
      const double sy = h->red_host[0], ss = h->red_host[1];
      std::swap(u, u1);
      std::swap(g, g1);
      E = En;
      gn = std::sqrt(gsqn);
      if (step < tol) break;
      alpha = sy > 0 ? ss / sy : 2.0 * alpha;
    }
    k_total += k;
  }
  // the planes hold float32(u) of the last evaluation, the accepted iterate:
  // hand it back and install it as the gate's field (gather-window set-up
  // and check)
  for (int pl = 0; pl < 2; ++pl) {
    hipLaunchKernelGGL(k_from_padded<float>, grid, block, 0, h->stream, n, h->pitch, fP + pl * h->padded,
                       field + pl * n2);
    LAUNCH_OK();
  }
  if (loss) *loss = E;
  if (steps) *steps = k_total;
  mcr_motion m{};
  m.kind = MCR_MOTION_FIELD;
  m.field = field;
  return mcr_set_motion(h, gate, &m);
}

// ---------------------------------------------------------------------------
// Operators
// ---------------------------------------------------------------------------
template <typename T>
mcr_status apply_Ai_impl(mcr_handle* h, int gate, const void* x, void* out) {
  STATUS_OK(launch_warp<T>(h, gate, 1, (const T*)x));
  return launch_project<T, 0>(h, gate, 1, (T*)out, h->sino);
}

template <typename T>
mcr_status apply_Ai_adjoint_impl(mcr_handle* h, int gate, const void* s, void* out) {
  Work<T>& w = work<T>(h);
  STATUS_OK(launch_backproject<T>(h, 1, (const T*)s, h->sino, w.bP, h->padded, 1));
  return launch_twarp<T, 0>(h, gate, 1, (T*)out, UpdateArgs<T>{});
}

template <typename T>
mcr_status warp_impl(mcr_handle* h, int gate, const void* x, void* out) {
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  STATUS_OK(launch_warp<T>(h, gate, 1, (const T*)x));
  hipLaunchKernelGGL(k_from_padded<T>, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0, h->stream, n,
                     h->pitch, w.wP, (T*)out);
  LAUNCH_OK();
  return MCR_OK;
}

template <typename T>
mcr_status warp_adjoint_impl(mcr_handle* h, int gate, const void* b, void* out) {
  Work<T>& w = work<T>(h);
  const int n = h->geo.n;
  hipLaunchKernelGGL((k_to_padded<T, T>), dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0, h->stream, n,
                     h->pitch, (const T*)b, w.bP);
  LAUNCH_OK();
  return launch_twarp<T, 0>(h, gate, 1, (T*)out, UpdateArgs<T>{});
}

// ---------------------------------------------------------------------------
// FP64 diagnostics (always on the double workspace)
// ---------------------------------------------------------------------------
// out = sum over gates in [gate0, gate0+G) of A_g^* A_g v  (v unpadded double)
mcr_status normal_op64(mcr_handle* h, int gate0, int G, const double* v, double* out, int subset = -1) {
  Work<double>& w = h->wd;
  STATUS_OK(launch_warp<double>(h, gate0, G, v));
  STATUS_OK((launch_project<double, 0>(h, gate0, G, w.dy, h->sino, nullptr, subset)));
  STATUS_OK(launch_backproject<double>(h, G, w.dy, h->sino, w.bP, h->padded, 1, subset));
  return launch_twarp<double, 0>(h, gate0, G, out, UpdateArgs<double>{});
}

template <typename T>
mcr_status objective_impl(mcr_handle* h, const void* x, const void* const* d, double alpha, double* out) {
  STATUS_OK(init_work<double>(h));
  Work<double>& w = h->wd;
  const long n2 = (long)h->geo.n * h->geo.n;
  const int N = h->N;
  double* x64 = w.img;
  hipLaunchKernelGGL((k_convert<T, double>), dim3(cdiv(n2, 256)), dim3(256), 0, h->stream, n2,
                     (const T*)x, x64);
  LAUNCH_OK();
  STATUS_OK((launch_reduce<double, double, 0>(h, n2, x64, x64, 0)));
  STATUS_OK(read_results(h, 1));
  const double xx = h->red_host[0];
  // chunks of up to 32 gates share one warp and one projection launch;
  // each gate's residual norm goes to result slot 1 + (gate - g0)
  double resid = 0.0;
  const int chunk = std::min(32, h->nslots);
  for (int g0 = 0; g0 < N; g0 += chunk) {
    const int G = std::min(chunk, N - g0);
    STATUS_OK(launch_warp<double>(h, g0, G, x64));
    STATUS_OK((launch_project<double, 0>(h, g0, G, w.dy, h->sino)));
    for (int i = 0; i < G; ++i)
      STATUS_OK((launch_reduce<double, T, 2>(h, h->sino, w.dy + i * h->sino, (const T*)d[g0 + i], 1 + i)));
    STATUS_OK(read_results(h, 1 + G));
    for (int i = 0; i < G; ++i) resid += h->red_host[1 + i];
  }
  const double val = alpha * xx + resid / N;
  if (!std::isfinite(val)) return fail(MCR_ERR_NONFINITE, "objective is not finite");
  *out = val;
  return MCR_OK;
}

template <typename T>
mcr_status gap_impl(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha, double* out) {
  double obj = 0.0;
  STATUS_OK(objective_impl<T>(h, st->x, d, alpha, &obj));
  Work<double>& w = h->wd;
  const int N = h->N;
  const long n2 = (long)h->geo.n * h->geo.n;
  // z = sum_i A_i^* y_i in FP64, 32 gates per launch, accumulated into img2
  double dual = 0.0;
  const int chunk = std::min(32, h->nslots);
  for (int g0 = 0; g0 < N; g0 += chunk) {
    const int G = std::min(chunk, N - g0);
    for (int i = 0; i < G; ++i) {
      hipLaunchKernelGGL((k_convert<T, double>), dim3(cdiv(h->sino, 256)), dim3(256), 0, h->stream, h->sino,
                         (const T*)st->y[g0 + i], w.dy + i * h->sino);
      LAUNCH_OK();
    }
    STATUS_OK(launch_backproject<double>(h, G, w.dy, h->sino, w.bP, h->padded, 1));
    if (g0 == 0)
      STATUS_OK((launch_twarp<double, 0>(h, g0, G, w.img2, UpdateArgs<double>{})));
    else
      STATUS_OK((launch_twarp<double, 1>(h, g0, G, w.img2, UpdateArgs<double>{})));
    for (int i = 0; i < G; ++i) {
      STATUS_OK((launch_reduce<T, T, 1>(h, h->sino, (const T*)st->y[g0 + i], (const T*)d[g0 + i], 2 * i)));
      STATUS_OK((launch_reduce<T, T, 0>(h, h->sino, (const T*)st->y[g0 + i], (const T*)st->y[g0 + i], 2 * i + 1)));
    }
    STATUS_OK(read_results(h, 2 * G));
    for (int i = 0; i < G; ++i) dual += h->red_host[2 * i] + 0.25 * N * h->red_host[2 * i + 1];
  }
  STATUS_OK((launch_reduce<double, double, 0>(h, n2, w.img2, w.img2, 0)));
  STATUS_OK(read_results(h, 1));
  const double val = obj + h->red_host[0] / (4.0 * alpha) + dual;
  if (!std::isfinite(val)) return fail(MCR_ERR_NONFINITE, "duality gap is not finite");
  *out = val;
  return MCR_OK;
}

}  // namespace

namespace {

// One SPDHG epoch of every slice of a batch: step (i) for all slices, then for
// each round t the four phases over the round's slots (one launch each, block
// z = slot; a slot is one iteration of one slice). Kernels read gates, slices and per-slice scalars from
// device tables, so the launch sequence does not depend on the gate draws and
// can be replayed as a graph.
template <typename T>
mcr_status batch_launches(mcr_handle* h, T* x, T* z, T* zbar) {
  Work<T>& w = work<T>(h);
  mcr_handle::Batch& B = h->batch;
  const long n2 = (long)h->geo.n * h->geo.n;
  const T* tc = (const T*)B.tc;
  {
    Timed tm(h, MCR_KERNEL_XSTEP);
    hipLaunchKernelGGL(k_xstep_batch<T>, dim3(cdiv(n2, 256), B.S), dim3(256), 0, h->stream, n2, x, zbar, tc);
    LAUNCH_OK();
  }
  for (int t = 0; t < B.tmax; ++t) {
    const int cnt = B.nact[t];
    const SlotInfo* sl = B.slots + (long)t * B.S;
    STATUS_OK(launch_warp<T>(h, 0, cnt, x, sl, n2));
    STATUS_OK((launch_project<T, 1>(h, 0, cnt, w.dy, h->sino, sl)));
    STATUS_OK(launch_backproject<T>(h, cnt, w.dy, h->sino, w.bP, h->padded, 1));
    STATUS_OK((launch_twarp<T, 2>(h, 0, 1, nullptr, UpdateArgs<T>{x, z, zbar, T(0), T(0), 0}, sl, cnt, tc,
                                  max_radius(h, 0, h->N))));
  }
  return MCR_OK;
}

template <typename T>
mcr_status batch_epoch_impl(mcr_handle* h, void* x, void* z, void* zbar, void* y, const void* d,
                            const double* alpha, const double* sigma, const double* tau, const double* theta,
                            const double* p, const int32_t* seq, int use_graph) {
  mcr_handle::Batch& B = h->batch;
  const int N = h->N, S = B.S;
  // per-gate scalars and pointers (slice s has N_s gates, serial sampling p)
  std::vector<GateScalars<T>> sc(N);
  std::vector<GatePtrs<T>> pt(N);
  for (int s = 0; s < S; ++s) {
    for (int k = 0; k < B.ng[s]; ++k) {
      const int gid = B.off[s] + k;
      sc[gid].sigma = T(sigma[gid]);
      sc[gid].cy = T(1.0 / (1.0 + sigma[gid] * B.ng[s] / 2.0));
      sc[gid].coef = T(theta[s] / p[gid]);
      sc[gid].pad_ = T(0);
      pt[gid].y = (T*)y + (long)gid * h->sino;
      pt[gid].d = (const T*)d + (long)gid * h->sino;
    }
  }
  Work<T>& w = work<T>(h);
  w.sc_host = sc;
  w.pt_host = pt;
  STATUS_OK(upload_params<T>(h, sc, pt));
  // slot tables of this epoch's draws and the slices' (tau, c_x)
  const size_t slot_bytes = sizeof(SlotInfo) * (size_t)B.tmax * S;
  if (B.pin_recorded) HIP_OK(hipEventSynchronize(B.pin_ev));
  SlotInfo* hs = (SlotInfo*)B.pin;
  for (int t = 0; t < B.tmax; ++t) {
    int c = 0;
    for (int q = B.round_off[t]; q < B.round_off[t + 1]; ++q, ++c) {
      const int s = B.items[q].x, j = B.items[q].y;
      hs[(long)t * S + c] = SlotInfo{s, B.off[s] + seq[B.off[s] + j], j + 1 < B.ng[s] ? 1 : 0, 0};
    }
    for (; c < S; ++c) hs[(long)t * S + c] = SlotInfo{0, 0, 0, 0};
  }
  T* htc = (T*)((char*)B.pin + slot_bytes);
  for (int s = 0; s < S; ++s) {
    htc[2 * s] = T(tau[s]);
    htc[2 * s + 1] = T(1.0 / (1.0 + 2.0 * tau[s] * alpha[s]));
  }
  HIP_OK(hipMemcpyAsync(B.slots, B.pin, slot_bytes, hipMemcpyHostToDevice, h->stream));
  HIP_OK(hipMemcpyAsync(B.tc, htc, sizeof(T) * 2 * S, hipMemcpyHostToDevice, h->stream));
  HIP_OK(hipEventRecord(B.pin_ev, h->stream));
  B.pin_recorded = true;
  if (!use_graph) return batch_launches<T>(h, (T*)x, (T*)z, (T*)zbar);
  // graph: captured once per (x, z, zbar) and handle configuration (variants,
  // window radii) on the batch stream, replayed on the handle's stream
  if (!B.exec || B.key[0] != x || B.key[1] != z || B.key[2] != zbar || B.gen != h->config_gen) {
    if (B.exec) {
      HIP_OK(hipStreamSynchronize(h->stream));  // the previous replay may still run
      (void)hipGraphExecDestroy(B.exec);
      B.exec = nullptr;
    }
    if (B.graph) {
      (void)hipGraphDestroy(B.graph);
      B.graph = nullptr;
    }
    hipStream_t caller = h->stream;
    const bool prof = h->prof;
    h->prof = false;
    h->stream = B.gstream;
    HIP_OK(hipStreamBeginCapture(B.gstream, hipStreamCaptureModeThreadLocal));
    mcr_status st = batch_launches<T>(h, (T*)x, (T*)z, (T*)zbar);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(B.gstream, &g);
    h->stream = caller;
    h->prof = prof;
    if (st != MCR_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(MCR_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    B.graph = g;
    HIP_OK(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    B.key[0] = x;
    B.key[1] = z;
    B.key[2] = zbar;
    B.gen = h->config_gen;
  }
  // the replay itself goes on the handle's stream (a graph can be launched
  // on the null stream, only captured off it), after the table uploads
  {
    Timed tm(h, MCR_KERNEL_OTHER);
    HIP_OK(hipGraphLaunch(B.exec, h->stream));
  }
  return MCR_OK;
}

}  // namespace

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, mcr_handle::Tune> g_tune_cache;

// Average duration [ms] of `reps` launches made by fn after two warm-up launches.
template <typename F>
mcr_status time_launches(mcr_handle* h, F fn, int reps, float* ms) {
  hipEvent_t a, b;
  HIP_OK(hipEventCreate(&a));
  HIP_OK(hipEventCreate(&b));
  mcr_status st = MCR_OK;
  for (int i = 0; i < 2 && st == MCR_OK; ++i) st = fn();
  if (st == MCR_OK) {
    (void)hipEventRecord(a, h->stream);
    for (int i = 0; i < reps && st == MCR_OK; ++i) st = fn();
    (void)hipEventRecord(b, h->stream);
    (void)hipEventSynchronize(b);
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, a, b);
    *ms = t / reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return st;
}
}  // namespace

namespace {
mcr_status create_impl(const mcr_geometry* geom, int32_t n_gates, const mcr_motion* motion, mcr_dtype dtype,
                       void* stream, int nslots, mcr_handle** out);
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* mcr_last_error(void) { return g_err.c_str(); }

mcr_status mcr_create(const mcr_geometry* geom, int32_t n_gates, const mcr_motion* motion, mcr_dtype dtype,
                      void* stream, mcr_handle** out) {
  return create_impl(geom, n_gates, motion, dtype, stream, 0, out);
}

}  // extern "C"

namespace {
mcr_status create_impl(const mcr_geometry* geom, int32_t n_gates, const mcr_motion* motion, mcr_dtype dtype,
                       void* stream, int nslots, mcr_handle** out) {
  if (!out) return fail(MCR_ERR_ARG, "out is null");
  *out = nullptr;
  if (!geom) return fail(MCR_ERR_ARG, "geometry is null");
  if (geom->n < 1 || geom->n > 4096) return fail(MCR_ERR_ARG, "n = %d must be in [1, 4096]", geom->n);
  if (geom->n_angles < 1 || geom->n_angles > 16384)
    return fail(MCR_ERR_ARG, "n_angles = %d must be in [1, 16384]", geom->n_angles);
  if (geom->n_det < 1 || geom->n_det > 16384)
    return fail(MCR_ERR_ARG, "n_det = %d must be in [1, 16384]", geom->n_det);
  if (n_gates < 1 || n_gates > 4096) return fail(MCR_ERR_ARG, "n_gates = %d must be in [1, 4096]", n_gates);
  if (!motion) return fail(MCR_ERR_ARG, "motion is null");
  for (int i = 0; i < n_gates; ++i) STATUS_OK(check_motion(&motion[i], i));
  if (dtype != MCR_F32 && dtype != MCR_F64) return fail(MCR_ERR_ARG, "unknown dtype %d", (int)dtype);

  mcr_handle* h = new mcr_handle();
  h->geo = *geom;
  h->N = n_gates;
  h->dtype = dtype;
  h->stream = (hipStream_t)stream;
  h->nslots = nslots > 0 ? std::min(nslots, (int)n_gates) : n_gates;
  h->pitch = geom->n + 2 * kPad;
  h->padded = (long)h->pitch * h->pitch;
  h->sino = (long)geom->n_angles * geom->n_det;
  h->motion.assign(motion, motion + n_gates);
  h->radius.assign(n_gates, 1);
  h->sub = {AngleRanges{0, geom->n_angles, 0, 0}};
  for (auto& m : h->motion) {
    if (m.kind == MCR_MOTION_FIELD) h->any_field = true;
  }
  auto cleanup = [&](mcr_status s) {
    mcr_destroy(h);
    return s;
  };
  mcr_status s;
  const int n = geom->n;
  if ((s = dmalloc(h, (void**)&h->fieldP, sizeof(float) * 2 * h->padded * (h->any_field ? n_gates : 1))) != MCR_OK)
    return cleanup(s);
  if ((s = dmalloc(h, (void**)&h->centres, sizeof(short2) * (long)n * n * (h->any_field ? n_gates : 1))) != MCR_OK)
    return cleanup(s);
  if ((s = dmalloc(h, (void**)&h->red_partial, sizeof(double) * kRedBlocks)) != MCR_OK) return cleanup(s);
  if ((s = dmalloc(h, (void**)&h->red_out, sizeof(double) * 64)) != MCR_OK) return cleanup(s);
  if ((s = dmalloc(h, (void**)&h->need, sizeof(int) * 4)) != MCR_OK) return cleanup(s);
  if ((s = dmalloc(h, (void**)&h->mgrad_partial, sizeof(double) * 3 * cdiv(n, 16) * cdiv(n, 16))) != MCR_OK)
    return cleanup(s);
  if (hipHostMalloc((void**)&h->red_host, sizeof(double) * 64, hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(MCR_ERR_NOMEM, "pinned allocation failed"));
  // copy fields into the padded layout and build the window centres
  for (int i = 0; i < n_gates && h->any_field; ++i) {
    if (h->motion[i].kind != MCR_MOTION_FIELD) continue;
    float* dst = h->fieldP + (long)i * 2 * h->padded;
    for (int pl = 0; pl < 2; ++pl) {
      hipLaunchKernelGGL((k_to_padded<float, float>), dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0,
                         h->stream, n, h->pitch, h->motion[i].field + (long)pl * n * n, dst + pl * h->padded);
    }
    hipLaunchKernelGGL(k_field_centres, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0, h->stream, n, h->pitch,
                       dst, h->padded, h->centres + (long)i * n * n);
    h->motion[i].field = nullptr;
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
    return cleanup(fail(MCR_ERR_HIP, "field set-up failed"));
  if ((s = init_work<double>(h)) != MCR_OK) return cleanup(s);
  if (dtype == MCR_F32 && (s = init_work<float>(h)) != MCR_OK) return cleanup(s);
  if ((s = mcr_set_motion(h, -1, nullptr)) != MCR_OK) return cleanup(s);
  // defaults before any autotuning: the quarter-turn pair where the geometry
  // has the symmetry, else the line-sheared forward and the tiled adjoint
  h->tune.fwd = h->qt[0].npieces > 0 ? 4 : (h->shear_npieces > 0 ? 3 : (h->sched_ok ? 2 : 0));
  const bool even = geom->n % 2 == 0 && geom->n_angles % 2 == 0;
  h->tune.adj_px = even ? -4 : 8;
  h->tune.adj_s = even ? 16 : 6;
  *out = h;
  return MCR_OK;
}
}  // namespace

extern "C" {

mcr_status mcr_destroy(mcr_handle* h) {
  if (!h) return MCR_OK;
  // release everything even if the runtime reports an earlier error
  (void)(h->stream ? hipStreamSynchronize(h->stream) : hipDeviceSynchronize());
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->red_host) (void)hipHostFree(h->red_host);
  if (h->wf.pin) (void)hipHostFree(h->wf.pin);
  if (h->wd.pin) (void)hipHostFree(h->wd.pin);
  if (h->wf.pin_ev) (void)hipEventDestroy(h->wf.pin_ev);
  if (h->wd.pin_ev) (void)hipEventDestroy(h->wd.pin_ev);
  for (auto& r : h->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : h->spare) (void)hipEventDestroy(e);
  if (h->mot_pin) (void)hipHostFree(h->mot_pin);
  if (h->mot_ev) (void)hipEventDestroy(h->mot_ev);
  if (h->batch.exec) (void)hipGraphExecDestroy(h->batch.exec);
  if (h->batch.graph) (void)hipGraphDestroy(h->batch.graph);
  if (h->batch.pin) (void)hipHostFree(h->batch.pin);
  if (h->batch.pin_ev) (void)hipEventDestroy(h->batch.pin_ev);
  if (h->batch.gstream) (void)hipStreamDestroy(h->batch.gstream);
  delete h;
  return MCR_OK;
}

mcr_status mcr_set_stream(mcr_handle* h, void* stream) {
  STATUS_OK(check_handle(h));
  HIP_OK(hipStreamSynchronize(h->stream));
  h->stream = (hipStream_t)stream;
  return MCR_OK;
}

// gate = -1 (internal): re-verify every gate's window with the current motion.
mcr_status mcr_set_motion(mcr_handle* h, int32_t gate, const mcr_motion* motion) {
  STATUS_OK(check_handle(h));
  const int n = h->geo.n;
  if (gate >= 0) {
    STATUS_OK(check_gate(h, gate));
    STATUS_OK(check_ptr(motion, "motion"));
    STATUS_OK(check_motion(motion, gate));
    if (motion->kind == MCR_MOTION_FIELD && !h->any_field)
      return fail(MCR_ERR_STATE, "handle was created without displacement fields");
    HIP_OK(hipStreamSynchronize(h->stream));
    h->motion[gate] = *motion;
    if (motion->kind == MCR_MOTION_FIELD) {
      float* dst = h->fieldP + (long)gate * 2 * h->padded;
      for (int pl = 0; pl < 2; ++pl) {
        hipLaunchKernelGGL((k_to_padded<float, float>), dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0,
                           h->stream, n, h->pitch, motion->field + (long)pl * n * n, dst + pl * h->padded);
        LAUNCH_OK();
      }
      hipLaunchKernelGGL(k_field_centres, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0, h->stream, n, h->pitch,
                         dst, h->padded, h->centres + (long)gate * n * n);
      LAUNCH_OK();
      h->motion[gate].field = nullptr;
    }
  }
  // verify the gather windows with both precisions' arithmetic
  const int g0 = gate >= 0 ? gate : 0, g1 = gate >= 0 ? gate + 1 : h->N;
  STATUS_OK(upload_motion<double>(h));
  if (h->wf.ready) STATUS_OK(upload_motion<float>(h));
  for (int i = g0; i < g1; ++i) {
    if (h->motion[i].kind == MCR_MOTION_IDENTITY) {
      h->radius[i] = 1;
      continue;
    }
    HIP_OK(hipMemsetAsync(h->need, 0, sizeof(int), h->stream));
    dim3 grid(cdiv(n, 16), cdiv(n, 16)), block(16, 16);
    hipLaunchKernelGGL(k_window_check<double>, grid, block, 0, h->stream, geo_of<double>(h), h->wd.motion, i,
                       h->fieldP, 2 * h->padded, h->padded, h->centres, h->need);
    LAUNCH_OK();
    if (h->wf.ready) {
      hipLaunchKernelGGL(k_window_check<float>, grid, block, 0, h->stream, geo_of<float>(h), h->wf.motion, i,
                         h->fieldP, 2 * h->padded, h->padded, h->centres, h->need);
      LAUNCH_OK();
    }
    int need = 0;
    HIP_OK(hipMemcpyAsync(&need, h->need, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    if (need > kMaxRadius) {
      // leave a consistent handle: the gate's field planes already hold the
      // rejected field, so the gate falls back to the identity
      STATUS_OK(reset_gate_identity(h, i));
      return fail(MCR_ERR_STATE,
                  "gate %d: the displacement field folds too strongly for a %dx%d transposed-warp window (needs %d); "
                  "the gate is reset to the identity",
                  i, 2 * kMaxRadius + 1, 2 * kMaxRadius + 1, need);
    }
    h->radius[i] = std::max(1, need);
  }
  ++h->config_gen;
  STATUS_OK(upload_motion<double>(h));
  if (h->wf.ready) STATUS_OK(upload_motion<float>(h));
  return MCR_OK;
}

// Rigid motion needs no window check. Output pixel p of the transposed warp
// gathers from the pixels q whose sample position R q + t lies within one
// pixel of p (per axis), i.e. q in R^T (p - t + (-1, 1)^2): per axis within
// |cos| + |sin| <= sqrt(2) of the exact inverse image c = R^T (p - t). Centred
// on round(c), every such q is within sqrt(2) + 1/2 < 2, hence (being integer)
// within 1: the 3 x 3 window holds them all.
mcr_status mcr_set_rigid_params(mcr_handle* h, const double* params) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_ptr(params, "params"));
  for (int i = 0; i < h->N; ++i) {
    if (h->motion[i].kind != MCR_MOTION_RIGID) return fail(MCR_ERR_STATE, "gate %d is not rigid", i);
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(params[3 * i + k])) return fail(MCR_ERR_ARG, "params[%d][%d] is not finite", i, k);
  }
  const size_t bd = sizeof(GateMotion<double>) * (h->N + 1), bf = sizeof(GateMotion<float>) * (h->N + 1);
  if (!h->mot_pin) {
    HIP_OK(hipHostMalloc(&h->mot_pin, bd + bf, hipHostMallocDefault));
    HIP_OK(hipEventCreateWithFlags(&h->mot_ev, hipEventDisableTiming));
  }
  if (h->mot_recorded) HIP_OK(hipEventSynchronize(h->mot_ev));
  for (int i = 0; i < h->N; ++i) {
    for (int k = 0; k < 3; ++k) h->motion[i].rigid[k] = params[3 * i + k];
    h->radius[i] = 1;
  }
  GateMotion<double>* md = (GateMotion<double>*)h->mot_pin;
  GateMotion<float>* mf = (GateMotion<float>*)((char*)h->mot_pin + bd);
  for (int i = 0; i <= h->N; ++i) {
    md[i] = gate_motion<double>(h, i);
    mf[i] = gate_motion<float>(h, i);
  }
  HIP_OK(hipMemcpyAsync(h->wd.motion, md, bd, hipMemcpyHostToDevice, h->stream));
  if (h->wf.ready) HIP_OK(hipMemcpyAsync(h->wf.motion, mf, bf, hipMemcpyHostToDevice, h->stream));
  HIP_OK(hipEventRecord(h->mot_ev, h->stream));
  h->mot_recorded = true;
  ++h->config_gen;
  return MCR_OK;
}

mcr_status mcr_get_info(const mcr_handle* h, mcr_geometry* geom, int32_t* n_gates, mcr_dtype* dtype,
                        int32_t* window_radius) {
  STATUS_OK(check_handle(h));
  if (geom) *geom = h->geo;
  if (n_gates) *n_gates = h->N;
  if (dtype) *dtype = h->dtype;
  if (window_radius) {
    int r = 1;
    for (int v : h->radius) r = std::max(r, v);
    *window_radius = r;
  }
  return MCR_OK;
}

#define DISPATCH(fn, ...) \
  (h->dtype == MCR_F32 ? fn<float>(__VA_ARGS__) : fn<double>(__VA_ARGS__))

mcr_status mcr_warp(mcr_handle* h, int32_t gate, const void* x, void* img) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_gate(h, gate));
  STATUS_OK(check_ptr(x, "x"));
  STATUS_OK(check_ptr(img, "img"));
  return DISPATCH(warp_impl, h, gate, x, img);
}

mcr_status mcr_warp_adjoint(mcr_handle* h, int32_t gate, const void* b, void* img) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_gate(h, gate));
  STATUS_OK(check_ptr(b, "b"));
  STATUS_OK(check_ptr(img, "img"));
  return DISPATCH(warp_adjoint_impl, h, gate, b, img);
}

mcr_status mcr_project(mcr_handle* h, const void* x, void* sino) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_ptr(x, "x"));
  STATUS_OK(check_ptr(sino, "sino"));
  return DISPATCH(apply_Ai_impl, h, h->N, x, sino);  // entry N of the motion table is the identity
}

mcr_status mcr_backproject(mcr_handle* h, const void* sino, void* img) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_ptr(sino, "sino"));
  STATUS_OK(check_ptr(img, "img"));
  if (h->dtype == MCR_F32)
    return launch_backproject<float>(h, 1, (const float*)sino, h->sino, (float*)img, 0, 0);
  return launch_backproject<double>(h, 1, (const double*)sino, h->sino, (double*)img, 0, 0);
}

mcr_status mcr_apply_Ai(mcr_handle* h, int32_t gate, const void* x, void* sino) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_gate(h, gate));
  STATUS_OK(check_ptr(x, "x"));
  STATUS_OK(check_ptr(sino, "sino"));
  return DISPATCH(apply_Ai_impl, h, gate, x, sino);
}

mcr_status mcr_apply_Ai_adjoint(mcr_handle* h, int32_t gate, const void* sino, void* img) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_gate(h, gate));
  STATUS_OK(check_ptr(sino, "sino"));
  STATUS_OK(check_ptr(img, "img"));
  return DISPATCH(apply_Ai_adjoint_impl, h, gate, sino, img);
}

mcr_status mcr_spdhg_iterate(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha,
                             const double* sigma, double tau, double theta, const double* p,
                             const int32_t* gate_seq, int32_t n_iter) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_alg(h, st, d, alpha, sigma, tau, theta, p));
  STATUS_OK(check_ptr(p, "p"));
  STATUS_OK(check_ptr(gate_seq, "gate_seq"));
  if (n_iter < 0) return fail(MCR_ERR_ARG, "n_iter = %d must be >= 0", n_iter);
  for (int k = 0; k < n_iter; ++k) STATUS_OK(check_gate(h, gate_seq[k]));
  if (n_iter == 0) return MCR_OK;
  return DISPATCH(spdhg_impl, h, st, d, alpha, sigma, tau, theta, p, gate_seq, n_iter);
}

mcr_status mcr_spdhg_epoch(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha,
                           const double* sigma, double tau, double theta, const double* p,
                           const int32_t* gate_seq) {
  STATUS_OK(check_handle(h));
  return mcr_spdhg_iterate(h, st, d, alpha, sigma, tau, theta, p, gate_seq, h->N);
}

mcr_status mcr_pdhg_epoch(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha,
                          const double* sigma, double tau, double theta) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_alg(h, st, d, alpha, sigma, tau, theta, nullptr));
  if (h->nslots < h->N) return fail(MCR_ERR_STATE, "PDHG over all gates is not available on a batch handle");
  return DISPATCH(pdhg_impl, h, st, d, alpha, sigma, tau, theta);
}

mcr_status mcr_spdhg_iterate_ckpt(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha,
                                  const double* sigma, double tau, double theta, const double* p,
                                  const int32_t* gate_seq, int32_t n_iter, void* const* x1_ckpt,
                                  void* const* y_ckpt, void* const* b_ckpt) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_alg(h, st, d, alpha, sigma, tau, theta, p));
  STATUS_OK(check_ptr(p, "p"));
  STATUS_OK(check_ptr(gate_seq, "gate_seq"));
  if (n_iter < 0) return fail(MCR_ERR_ARG, "n_iter = %d must be >= 0", n_iter);
  if (n_iter > 0) {
    STATUS_OK(check_ptr(x1_ckpt, "x1_ckpt"));
    STATUS_OK(check_ptr(y_ckpt, "y_ckpt"));
  }
  for (int k = 0; k < n_iter; ++k) {
    STATUS_OK(check_gate(h, gate_seq[k]));
    if (!x1_ckpt[k] || !y_ckpt[k] || (b_ckpt && !b_ckpt[k])) return fail(MCR_ERR_ARG, "checkpoint %d is null", k);
  }
  if (n_iter == 0) return MCR_OK;
  return DISPATCH(spdhg_ckpt_impl, h, st, d, alpha, sigma, tau, theta, p, gate_seq, n_iter, x1_ckpt, y_ckpt,
                  b_ckpt);
}

mcr_status mcr_spdhg_step_backward(mcr_handle* h, int32_t gate, const void* x1, const void* y_before,
                                   const void* d_gate, double alpha, double sigma, double tau, double theta,
                                   double p, void* gx, void* gy_gate, void* gz, void* gzbar, void* grad_motion,
                                   const void* b_ckpt) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_gate(h, gate));
  STATUS_OK(check_ptr(x1, "x1"));
  STATUS_OK(check_ptr(y_before, "y_before"));
  STATUS_OK(check_ptr(d_gate, "d_gate"));
  STATUS_OK(check_ptr(gx, "gx"));
  STATUS_OK(check_ptr(gy_gate, "gy_gate"));
  STATUS_OK(check_ptr(gz, "gz"));
  STATUS_OK(check_ptr(gzbar, "gzbar"));
  if (!(alpha > 0) || !std::isfinite(alpha)) return fail(MCR_ERR_ARG, "alpha = %g must be finite and > 0", alpha);
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(MCR_ERR_ARG, "sigma = %g must be finite and > 0", sigma);
  if (!(tau > 0) || !std::isfinite(tau)) return fail(MCR_ERR_ARG, "tau = %g must be finite and > 0", tau);
  if (!(theta >= 0) || !std::isfinite(theta)) return fail(MCR_ERR_ARG, "theta = %g must be finite and >= 0", theta);
  if (!(p > 0) || !(p <= 1)) return fail(MCR_ERR_ARG, "p = %g must be in (0, 1]", p);
  return DISPATCH(step_backward_impl, h, gate, x1, y_before, d_gate, alpha, sigma, tau, theta, p, gx, gy_gate, gz,
                  gzbar, grad_motion, b_ckpt);
}

mcr_status mcr_warp_motion_grad(mcr_handle* h, int32_t gate, const void* img, const void* v, void* grad_motion) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_gate(h, gate));
  STATUS_OK(check_ptr(img, "img"));
  STATUS_OK(check_ptr(v, "v"));
  STATUS_OK(check_ptr(grad_motion, "grad_motion"));
  return DISPATCH(motion_grad_impl, h, gate, img, v, grad_motion);
}

mcr_status mcr_register_affine(mcr_handle* h, int32_t gate, const void* ref, const void* target, double* params,
                               int32_t max_iter, double tol, double* loss, int32_t* steps) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_gate(h, gate));
  STATUS_OK(check_ptr(ref, "ref"));
  STATUS_OK(check_ptr(target, "target"));
  STATUS_OK(check_ptr(params, "params"));
  if (h->motion[gate].kind != MCR_MOTION_FIELD) return fail(MCR_ERR_ARG, "gate %d is not a field gate", gate);
  for (int m = 0; m < 6; ++m)
    if (!std::isfinite(params[m])) return fail(MCR_ERR_ARG, "params[%d] is not finite", m);
  if (max_iter < 0) return fail(MCR_ERR_ARG, "max_iter = %d must be >= 0", max_iter);
  if (!(tol >= 0) || !std::isfinite(tol)) return fail(MCR_ERR_ARG, "tol must be finite and >= 0");
  const mcr_status st = DISPATCH(register_affine_impl, h, gate, ref, target, params, max_iter, tol, loss, steps);
  if (st != MCR_OK && h->motion[gate].kind == MCR_MOTION_FIELD) {
    // the gate's planes hold an evaluated map whose windows were not set up
    const std::string msg = mcr_last_error();
    (void)reset_gate_identity(h, gate);
    return fail(st, "%s; the gate is reset to the identity", msg.c_str());
  }
  return st;
}

mcr_status mcr_register_field(mcr_handle* h, int32_t gate, const void* ref, const void* target, void* field,
                              double lambda, const double* sigmas, int32_t n_levels, int32_t max_iter, double tol,
                              double* loss, int32_t* steps) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_gate(h, gate));
  STATUS_OK(check_ptr(ref, "ref"));
  STATUS_OK(check_ptr(target, "target"));
  STATUS_OK(check_ptr(field, "field"));
  if (h->motion[gate].kind != MCR_MOTION_FIELD) return fail(MCR_ERR_ARG, "gate %d is not a field gate", gate);
  if (!(lambda >= 0) || !std::isfinite(lambda)) return fail(MCR_ERR_ARG, "lambda must be finite and >= 0");
  if (max_iter < 0) return fail(MCR_ERR_ARG, "max_iter = %d must be >= 0", max_iter);
  if (!(tol >= 0) || !std::isfinite(tol)) return fail(MCR_ERR_ARG, "tol must be finite and >= 0");
  if (n_levels < 0 || n_levels > kMaxLevels)
    return fail(MCR_ERR_ARG, "n_levels = %d must be in [0, %d]", n_levels, kMaxLevels);
  if (n_levels > 0) {
    STATUS_OK(check_ptr(sigmas, "sigmas"));
    for (int l = 0; l < n_levels; ++l)
      if (!(sigmas[l] >= 0 && sigmas[l] <= kMaxBlurSigma))
        return fail(MCR_ERR_ARG, "sigmas[%d] must be in [0, %g]", l, kMaxBlurSigma);
  }
  const mcr_status st = DISPATCH(register_field_impl, h, gate, ref, target, (float*)field, lambda, sigmas, n_levels,
                                 max_iter, tol, loss, steps);
  if (st != MCR_OK && h->motion[gate].kind == MCR_MOTION_FIELD) {
    // the gate's planes hold an evaluated map whose windows were not set up
    const std::string msg = mcr_last_error();
    (void)reset_gate_identity(h, gate);
    return fail(st, "%s; the gate is reset to the identity", msg.c_str());
  }
  return st;
}

mcr_status mcr_register_rigid(mcr_handle* h, int32_t gate, const void* ref, const void* target, double* params,
                              int32_t max_iter, double tol, double* loss, int32_t* steps) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_gate(h, gate));
  STATUS_OK(check_ptr(ref, "ref"));
  STATUS_OK(check_ptr(target, "target"));
  STATUS_OK(check_ptr(params, "params"));
  if (h->motion[gate].kind != MCR_MOTION_RIGID) return fail(MCR_ERR_ARG, "gate %d is not rigid", gate);
  for (int m = 0; m < 3; ++m)
    if (!std::isfinite(params[m])) return fail(MCR_ERR_ARG, "params[%d] is not finite", m);
  if (max_iter < 0) return fail(MCR_ERR_ARG, "max_iter = %d must be >= 0", max_iter);
  if (!(tol >= 0) || !std::isfinite(tol)) return fail(MCR_ERR_ARG, "tol must be finite and >= 0");
  return DISPATCH(register_rigid_impl, h, gate, ref, target, params, max_iter, tol, loss, steps);
}

}  // extern "C"

namespace {
mcr_status power_norm_impl(mcr_handle* h, int32_t gate, int subset, const double* v0, int32_t max_iter,
                           double rtol, double* out, int32_t* iters) {
  STATUS_OK(check_ptr(v0, "v0"));
  STATUS_OK(check_ptr(out, "out"));
  if (max_iter < 1) return fail(MCR_ERR_ARG, "max_iter = %d must be >= 1", max_iter);
  if (!(rtol >= 0) || !std::isfinite(rtol)) return fail(MCR_ERR_ARG, "rtol must be finite and >= 0");
  STATUS_OK(init_work<double>(h));
  Work<double>& w = h->wd;
  const long n2 = (long)h->geo.n * h->geo.n;
  double* v = w.img;
  double* av = w.img2;
  HIP_OK(hipMemcpyAsync(v, v0, sizeof(double) * n2, hipMemcpyDeviceToDevice, h->stream));
  STATUS_OK((launch_reduce<double, double, 0>(h, n2, v, v, 0)));
  STATUS_OK(read_results(h, 1));
  if (!(h->red_host[0] > 0)) return fail(MCR_ERR_ARG, "v0 must be nonzero and finite");
  double scale = 1.0 / std::sqrt(h->red_host[0]);
  double lam = 0.0;
  int it = 0;
  const int gate0 = gate < 0 ? 0 : gate, G = gate < 0 ? h->N : 1;
  for (it = 1; it <= max_iter; ++it) {
    hipLaunchKernelGGL(k_scale<double>, dim3(cdiv(n2, 256)), dim3(256), 0, h->stream, n2, v, scale);
    LAUNCH_OK();
    STATUS_OK(normal_op64(h, gate0, G, v, av, subset));
    STATUS_OK((launch_reduce<double, double, 1>(h, n2, v, av, 0)));
    STATUS_OK((launch_reduce<double, double, 0>(h, n2, av, av, 1)));
    STATUS_OK(read_results(h, 2));
    const double lam_new = h->red_host[0], nw2 = h->red_host[1];
    if (!std::isfinite(lam_new) || !std::isfinite(nw2)) return fail(MCR_ERR_NONFINITE, "power iteration diverged");
    if (nw2 == 0.0) {
      lam = 0.0;
      break;
    }
    std::swap(v, av);  // v <- A^*A v, rescaled at the top of the next iteration
    scale = 1.0 / std::sqrt(nw2);
    const bool done = it > 1 && std::fabs(lam_new - lam) <= rtol * std::fabs(lam_new);
    lam = lam_new;
    if (done) break;
  }
  HIP_OK(hipStreamSynchronize(h->stream));
  *out = lam;
  if (iters) *iters = std::min(it, max_iter);
  return MCR_OK;
}
}  // namespace

extern "C" {

mcr_status mcr_power_norm_sq(mcr_handle* h, int32_t gate, const double* v0, int32_t max_iter, double rtol,
                             double* out, int32_t* iters) {
  STATUS_OK(check_handle(h));
  if (gate != -1) STATUS_OK(check_gate(h, gate));
  if (gate == -1 && h->nslots < h->N)
    return fail(MCR_ERR_STATE, "the stacked norm over all gates is not available on a batch handle");
  return power_norm_impl(h, gate, -1, v0, max_iter, rtol, out, iters);
}

mcr_status mcr_block_norm_sq(mcr_handle* h, int32_t gate, int32_t subset, const double* v0, int32_t max_iter,
                             double rtol, double* out, int32_t* iters) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_gate(h, gate));
  if (subset < 0 || subset >= h->M) return fail(MCR_ERR_ARG, "subset = %d must be in [0, %d)", subset, h->M);
  return power_norm_impl(h, gate, subset, v0, max_iter, rtol, out, iters);
}

mcr_status mcr_set_subset_partition(mcr_handle* h, int32_t n_subsets, int32_t paired) {
  STATUS_OK(check_handle(h));
  const int na = h->geo.n_angles;
  if (paired && na % 2) return fail(MCR_ERR_ARG, "paired subsets need an even number of angles (n_angles = %d)", na);
  const int cap = paired ? na / 2 : na;
  if (n_subsets < 1 || n_subsets > cap)
    return fail(MCR_ERR_ARG, "n_subsets = %d must be in [1, %d]", n_subsets, cap);
  if (h->nslots < h->N) return fail(MCR_ERR_STATE, "angle subsets are not available on a batch handle");
  const bool pd = paired != 0 && n_subsets > 1;
  if (n_subsets == h->M && pd == h->sub_paired) return MCR_OK;
  HIP_OK(hipStreamSynchronize(h->stream));
  h->M = n_subsets;
  h->sub_paired = pd;
  h->sub.resize(n_subsets);
  const int H = na / 2;
  for (int s = 0; s < n_subsets; ++s) {
    if (pd) {
      const int a = (int)((long)s * H / n_subsets), b = (int)((long)(s + 1) * H / n_subsets);
      h->sub[s] = AngleRanges{a, b, a + H, b + H};
    } else {
      h->sub[s] = AngleRanges{(int)((long)s * na / n_subsets), (int)((long)(s + 1) * na / n_subsets), 0, 0};
    }
  }
  STATUS_OK(ensure_scalars<float>(h));
  STATUS_OK(ensure_scalars<double>(h));
  if (h->wf.ready) {
    const std::vector<AngleFx> af = angle_table_fx(h->geo.n, na, h->geo.n_det);
    STATUS_OK(upload_shear(h, af));
    STATUS_OK(upload_quad(h, af));
  }
  ++h->config_gen;
  return MCR_OK;
}

mcr_status mcr_set_subsets(mcr_handle* h, int32_t n_subsets) {
  return mcr_set_subset_partition(h, n_subsets, 0);
}

mcr_status mcr_spdhg_blocks_iterate(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha,
                                    const double* sigma, double tau, double theta, const double* p,
                                    const int32_t* block_seq, int32_t n_iter) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_alg(h, st, d, alpha, sigma, tau, theta, nullptr));
  STATUS_OK(check_ptr(p, "p"));
  STATUS_OK(check_ptr(block_seq, "block_seq"));
  const int nb = h->N * h->M;
  for (int b = 0; b < nb; ++b) {
    if (!(sigma[b] > 0) || !std::isfinite(sigma[b]))
      return fail(MCR_ERR_ARG, "sigma[%d] = %g must be finite and > 0", b, sigma[b]);
    if (!(p[b] > 0) || !(p[b] <= 1)) return fail(MCR_ERR_ARG, "p[%d] = %g must be in (0, 1]", b, p[b]);
  }
  if (n_iter < 0) return fail(MCR_ERR_ARG, "n_iter = %d must be >= 0", n_iter);
  for (int k = 0; k < n_iter; ++k)
    if (block_seq[k] < 0 || block_seq[k] >= nb)
      return fail(MCR_ERR_ARG, "block_seq[%d] = %d must be in [0, %d)", k, block_seq[k], nb);
  if (n_iter == 0) return MCR_OK;
  if (h->dtype == MCR_F32) STATUS_OK(init_work<float>(h));
  else STATUS_OK(init_work<double>(h));
  STATUS_OK(ensure_scalars<float>(h));
  STATUS_OK(ensure_scalars<double>(h));
  return DISPATCH(spdhg_blocks_impl, h, st, d, alpha, sigma, tau, theta, p, block_seq, n_iter);
}

mcr_status mcr_objective(mcr_handle* h, const void* x, const void* const* d, double alpha, double* out) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_ptr(x, "x"));
  STATUS_OK(check_ptr(d, "d"));
  STATUS_OK(check_ptr(out, "out"));
  for (int i = 0; i < h->N; ++i)
    if (!d[i]) return fail(MCR_ERR_ARG, "d[%d] is null", i);
  if (!(alpha > 0) || !std::isfinite(alpha)) return fail(MCR_ERR_ARG, "alpha must be finite and > 0");
  return DISPATCH(objective_impl, h, x, d, alpha, out);
}

mcr_status mcr_duality_gap(mcr_handle* h, const mcr_state* st, const void* const* d, double alpha, double* out) {
  STATUS_OK(check_handle(h));
  STATUS_OK(check_ptr(out, "out"));
  if (!st) return fail(MCR_ERR_ARG, "state is null");
  STATUS_OK(check_ptr(st->x, "state.x"));
  STATUS_OK(check_ptr(st->y, "state.y"));
  STATUS_OK(check_ptr(d, "d"));
  for (int i = 0; i < h->N; ++i) {
    if (!st->y[i]) return fail(MCR_ERR_ARG, "state.y[%d] is null", i);
    if (!d[i]) return fail(MCR_ERR_ARG, "d[%d] is null", i);
  }
  if (!(alpha > 0) || !std::isfinite(alpha)) return fail(MCR_ERR_ARG, "alpha must be finite and > 0");
  return DISPATCH(gap_impl, h, st, d, alpha, out);
}


namespace {
bool fwd_variant_ok(const mcr_handle* h, int f) {
  return f == 0 || (f == 1 && h->fwd_lds_ok) || (f == 2 && h->sched_ok) || (f == 3 && h->shear_npieces > 0) ||
         (f == 4 && h->qt[0].npieces > 0) || (f == 5 && h->qt[1].npieces > 0);
}
}  // namespace

mcr_status mcr_autotune(mcr_handle* h, int32_t gates_per_launch, int32_t* fwd, int32_t* adj_px, int32_t* adj_s) {
  STATUS_OK(check_handle(h));
  if (gates_per_launch < 1 || gates_per_launch > h->nslots)
    return fail(MCR_ERR_ARG, "gates_per_launch = %d must be in [1, %d] (the gates one launch of this handle covers)",
                gates_per_launch, h->nslots);
  if (h->dtype == MCR_F32) {
    const auto key = std::make_tuple(h->geo.n, h->geo.n_angles, h->geo.n_det, gates_per_launch);
    bool cached = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        h->tune = it->second;
        cached = true;
      }
    }
    if (!cached) {
      HIP_OK(hipStreamSynchronize(h->stream));
      const bool prof = h->prof;
      h->prof = false;
      Work<float>& w = h->wf;
      const int G = gates_per_launch;
      mcr_handle::Tune best = h->tune;
      mcr_status st = MCR_OK;
      // each variant is timed in two rounds over all candidates and keeps its
      // faster round (the first round also brings the GPU to its sustained
      // clocks, which otherwise favours the candidates timed last); the first
      // one (in the order below) within 3% of the fastest is kept, so that
      // near-ties resolve the same way run to run
      constexpr int kRounds = 2;
      auto pick = [](const std::vector<float>& t) {
        const float lo = *std::min_element(t.begin(), t.end());
        for (size_t i = 0; i < t.size(); ++i)
          if (t[i] <= 1.03f * lo) return (int)i;
        return 0;
      };
      // the forwards in order of preference; each is timed with the warp in
      // front of it, since the warp writes the planes the forward reads
      // (three quarter turns for 4, a transposed copy for the others).
      // Variant 5 is not a candidate: timed this way it won at 256^2 with 40
      // gates per launch, yet the batched epochs ran 2% slower with it than
      // with 4 (and 4% at 512^2 with one gate); mcr_set_variant selects it
      std::vector<int> fv;
      for (int f : {4, 3, 2, 1, 0})
        if (fwd_variant_ok(h, f)) fv.push_back(f);
      std::vector<float> ft(fv.size(), 1e30f);
      for (int r = 0; r < kRounds; ++r) {
        for (size_t i = 0; i < fv.size() && st == MCR_OK; ++i) {
          h->tune.fwd = fv[i];
          float ms = 0.0f;
          st = time_launches(h,
                             [&] {
                               STATUS_OK(launch_warp<float>(h, 0, G, w.img));
                               return launch_project<float, 0>(h, 0, G, w.dy, h->sino);
                             },
                             5, &ms);
          if (st == MCR_OK) ft[i] = std::min(ft[i], ms);
        }
      }
      if (st == MCR_OK && !fv.empty()) best.fwd = fv[pick(ft)];
      h->tune.fwd = best.fwd;
      // quarter-turn kernels first (tiled ones where the geometry has no
      // quarter-turn symmetry: they then run as their tiled counterparts)
      const int cand[][2] = {{-4, 16}, {-4, 8}, {-4, 12}, {-16, 8}, {-16, 16}, {-32, 16}, {-8, 16}, {-2, 8},
                             {8, 6}, {8, 8}, {8, 4}, {4, 4}, {4, 6}, {4, 8}, {4, 2}, {4, 1}, {2, 2}, {2, 1}, {1, 1},
                             {0, 1}};
      const int nc = (int)(sizeof(cand) / sizeof(cand[0]));
      std::vector<float> at(nc, 1e30f);
      for (int r = 0; r < kRounds; ++r) {
        for (int i = 0; i < nc && st == MCR_OK; ++i) {
          h->tune.adj_px = cand[i][0];
          h->tune.adj_s = cand[i][1];
          float ms = 0.0f;
          st = time_launches(h, [&] { return launch_backproject<float>(h, G, w.dy, h->sino, w.bP, h->padded, 1); },
                             5, &ms);
          if (st == MCR_OK) at[i] = std::min(at[i], ms);
        }
      }
      if (st == MCR_OK) {
        const int a = pick(at);
        best.adj_px = cand[a][0];
        best.adj_s = cand[a][1];
      }
      h->prof = prof;
      h->tune = best;
      STATUS_OK(st);
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[key] = best;
    }
  }
  ++h->config_gen;
  if (fwd) *fwd = h->tune.fwd;
  if (adj_px) *adj_px = h->tune.adj_px;
  if (adj_s) *adj_s = h->tune.adj_s;
  return MCR_OK;
}

mcr_status mcr_set_variant(mcr_handle* h, int32_t fwd, int32_t adj_px, int32_t adj_s) {
  STATUS_OK(check_handle(h));
  if (fwd < 0 || fwd > 5) return fail(MCR_ERR_ARG, "forward variant %d must be 0, 1, 2, 3, 4 or 5", fwd);
  if (h->dtype == MCR_F32 && fwd == 4 && (h->geo.n % 2 || h->geo.n_angles % 2))
    return fail(MCR_ERR_STATE, "the quarter-turn forward needs an even n and n_angles: its tables do not fit this "
                               "geometry");
  if (h->dtype == MCR_F32 && fwd == 5 && (h->geo.n % 2 || h->geo.n_angles % 4))
    return fail(MCR_ERR_STATE, "the eight-plane forward needs an even n and n_angles a multiple of 4: its tables "
                               "do not fit this geometry");
  if (h->dtype == MCR_F32 && !fwd_variant_ok(h, fwd))
    return fail(MCR_ERR_STATE, "the tiled forward's band windows do not fit this geometry");
  if (adj_px != 0 && adj_px != 1 && adj_px != 2 && adj_px != 4 && adj_px != 8 && adj_px != -2 && adj_px != -4 &&
      adj_px != -8 && adj_px != -16 && adj_px != -32)
    return fail(MCR_ERR_ARG, "pixels per thread %d must be 0, 1, 2, 4, 8, -2, -4, -8, -16 or -32", adj_px);
  if (adj_s < 1 || adj_s > kMaxShares) return fail(MCR_ERR_ARG, "angle shares %d must be in [1, %d]", adj_s, kMaxShares);
  h->tune.fwd = fwd;
  h->tune.adj_px = adj_px;
  h->tune.adj_s = adj_s;
  ++h->config_gen;
  return MCR_OK;
}

mcr_status mcr_batch_create(const mcr_geometry* geom, int32_t n_slices, const int32_t* gates_per_slice,
                            const mcr_motion* motion, mcr_dtype dtype, void* stream, mcr_handle** out) {
  if (!out) return fail(MCR_ERR_ARG, "out is null");
  *out = nullptr;
  if (n_slices < 1 || n_slices > 4096) return fail(MCR_ERR_ARG, "n_slices = %d must be in [1, 4096]", n_slices);
  STATUS_OK(check_ptr(gates_per_slice, "gates_per_slice"));
  long total = 0;
  int tmax = 0;
  for (int s = 0; s < n_slices; ++s) {
    if (gates_per_slice[s] < 1) return fail(MCR_ERR_ARG, "slice %d has %d gates", s, gates_per_slice[s]);
    total += gates_per_slice[s];
    tmax = std::max(tmax, (int)gates_per_slice[s]);
  }
  if (total > 4096) return fail(MCR_ERR_ARG, "%ld gates in total exceed 4096", total);
  mcr_handle* h = nullptr;
  STATUS_OK(create_impl(geom, (int)total, motion, dtype, stream, n_slices, &h));
  mcr_handle::Batch& B = h->batch;
  B.S = n_slices;
  B.ng.assign(gates_per_slice, gates_per_slice + n_slices);
  B.off.resize(n_slices);
  for (int s = 0, o = 0; s < n_slices; o += B.ng[s], ++s) B.off[s] = o;
  // rounds: an epoch takes tmax rounds (the longest slice's iterations);
  // slice s runs its iteration j in round floor(j tmax / N_s), so a slice's
  // iterations keep their order and every round holds about sum N_s / tmax
  // slots instead of all slices at the start and the longest ones alone at
  // the end
  B.tmax = tmax;
  B.nact.assign(tmax, 0);
  std::vector<std::vector<int2>> per_round(tmax);
  for (int s = 0; s < n_slices; ++s)
    for (int j = 0; j < B.ng[s]; ++j) per_round[(long)j * tmax / B.ng[s]].push_back(make_int2(s, j));
  B.items.clear();
  B.round_off.assign(tmax + 1, 0);
  for (int t = 0; t < tmax; ++t) {
    B.round_off[t] = (int)B.items.size();
    B.nact[t] = (int)per_round[t].size();
    B.items.insert(B.items.end(), per_round[t].begin(), per_round[t].end());
  }
  B.round_off[tmax] = (int)B.items.size();
  const size_t esz = dtype == MCR_F32 ? sizeof(float) : sizeof(double);
  const size_t slot_bytes = sizeof(SlotInfo) * (size_t)tmax * n_slices;
  mcr_status st = dmalloc(h, (void**)&B.slots, slot_bytes);
  if (st == MCR_OK) st = dmalloc(h, &B.tc, esz * 2 * n_slices);
  B.pin_bytes = slot_bytes + esz * 2 * n_slices;
  if (st == MCR_OK && hipHostMalloc(&B.pin, B.pin_bytes, hipHostMallocDefault) != hipSuccess)
    st = fail(MCR_ERR_NOMEM, "pinned allocation failed");
  if (st == MCR_OK && (hipEventCreateWithFlags(&B.pin_ev, hipEventDisableTiming) != hipSuccess ||
                       hipStreamCreateWithFlags(&B.gstream, hipStreamNonBlocking) != hipSuccess))
    st = fail(MCR_ERR_HIP, "could not create the batch stream and events");
  if (st == MCR_OK && hipStreamSynchronize(h->stream) != hipSuccess) st = fail(MCR_ERR_HIP, "batch set-up failed");
  if (st != MCR_OK) {
    mcr_destroy(h);
    return st;
  }
  *out = h;
  return MCR_OK;
}

mcr_status mcr_batch_spdhg_epoch(mcr_handle* h, void* x, void* z, void* zbar, void* y, const void* d,
                                 const double* alpha, const double* sigma, const double* tau, const double* theta,
                                 const double* p, const int32_t* gate_seq, int32_t use_graph) {
  STATUS_OK(check_handle(h));
  if (h->batch.S == 0) return fail(MCR_ERR_STATE, "not a batch handle (use mcr_batch_create)");
  STATUS_OK(check_ptr(x, "x"));
  STATUS_OK(check_ptr(z, "z"));
  STATUS_OK(check_ptr(zbar, "zbar"));
  STATUS_OK(check_ptr(y, "y"));
  STATUS_OK(check_ptr(d, "d"));
  STATUS_OK(check_ptr(alpha, "alpha"));
  STATUS_OK(check_ptr(sigma, "sigma"));
  STATUS_OK(check_ptr(tau, "tau"));
  STATUS_OK(check_ptr(theta, "theta"));
  STATUS_OK(check_ptr(p, "p"));
  STATUS_OK(check_ptr(gate_seq, "gate_seq"));
  const mcr_handle::Batch& B = h->batch;
  for (int s = 0; s < B.S; ++s) {
    if (!(alpha[s] > 0) || !std::isfinite(alpha[s])) return fail(MCR_ERR_ARG, "alpha[%d] must be finite and > 0", s);
    if (!(tau[s] > 0) || !std::isfinite(tau[s])) return fail(MCR_ERR_ARG, "tau[%d] must be finite and > 0", s);
    if (!(theta[s] >= 0) || !std::isfinite(theta[s])) return fail(MCR_ERR_ARG, "theta[%d] must be finite and >= 0", s);
    for (int k = 0; k < B.ng[s]; ++k) {
      const int gid = B.off[s] + k;
      if (!(sigma[gid] > 0) || !std::isfinite(sigma[gid])) return fail(MCR_ERR_ARG, "sigma[%d] must be finite and > 0", gid);
      if (!(p[gid] > 0) || !(p[gid] <= 1)) return fail(MCR_ERR_ARG, "p[%d] must be in (0, 1]", gid);
      if (gate_seq[gid] < 0 || gate_seq[gid] >= B.ng[s])
        return fail(MCR_ERR_ARG, "gate_seq[%d] = %d is not a gate of slice %d (it has %d)", gid, gate_seq[gid], s, B.ng[s]);
    }
  }
  return DISPATCH(batch_epoch_impl, h, x, z, zbar, y, d, alpha, sigma, tau, theta, p, gate_seq, use_graph);
}

mcr_status mcr_profile_enable(mcr_handle* h, int32_t enable) {
  STATUS_OK(check_handle(h));
  h->prof = enable != 0;
  return MCR_OK;
}

mcr_status mcr_profile_read(mcr_handle* h, double* total_ms, int64_t* launches) {
  STATUS_OK(check_handle(h));
  HIP_OK(hipStreamSynchronize(h->stream));
  double ms[MCR_KERNEL_CLASSES] = {0};
  int64_t cnt[MCR_KERNEL_CLASSES] = {0};
  for (auto& r : h->recs) {
    float t = 0.0f;
    HIP_OK(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.cls] += t;
    cnt[r.cls] += 1;
    h->spare.push_back(r.a);
    h->spare.push_back(r.b);
  }
  h->recs.clear();
  for (int i = 0; i < MCR_KERNEL_CLASSES; ++i) {
    if (total_ms) total_ms[i] = ms[i];
    if (launches) launches[i] = cnt[i];
  }
  return MCR_OK;
}

mcr_status mcr_step_sizes(int32_t algo, int32_t n_gates, const double* norms_sq, double alpha, double* sigma,
                          double* tau, double* theta, double* rate_per_epoch) {
  if (algo != 0 && algo != 1) return fail(MCR_ERR_ARG, "algo = %d must be 0 (SPDHG) or 1 (PDHG)", algo);
  if (n_gates < 1) return fail(MCR_ERR_ARG, "n_gates = %d must be >= 1", n_gates);
  STATUS_OK(check_ptr(norms_sq, "norms_sq"));
  STATUS_OK(check_ptr(sigma, "sigma"));
  if (!(alpha > 0) || !std::isfinite(alpha)) return fail(MCR_ERR_ARG, "alpha must be finite and > 0");
  const int cnt = algo == 0 ? n_gates : 1;
  for (int i = 0; i < cnt; ++i)
    if (!(norms_sq[i] > 0) || !std::isfinite(norms_sq[i]))
      return fail(MCR_ERR_ARG, "norms_sq[%d] = %g must be finite and > 0", i, norms_sq[i]);
  const double N = n_gates;
  if (algo == 0) {
    const double pr = 1.0 / N;
    double s = 0.0;
    for (int i = 0; i < n_gates; ++i) {
      const double si = std::sqrt(1.0 + norms_sq[i] / (alpha * N));
      s = std::max(s, si);
      sigma[i] = 2.0 / (N * (si - 1.0));
    }
    const double rho = 1.0 - 2.0 * pr / (1.0 + s);
    if (tau) *tau = pr / (2.0 * alpha * rho * (1.0 + s));
    if (theta) *theta = rho;
    if (rate_per_epoch) *rate_per_epoch = std::pow(rho, N);
  } else {
    const double s = std::sqrt(1.0 + norms_sq[0] / (alpha * N));
    for (int i = 0; i < n_gates; ++i) sigma[i] = 2.0 / (N * (s - 1.0));
    if (tau) *tau = 1.0 / (2.0 * alpha * (s - 1.0));
    if (theta) *theta = (s - 1.0) / (s + 1.0);
    if (rate_per_epoch) *rate_per_epoch = (s - 1.0) / (s + 1.0);
  }
  return MCR_OK;
}

mcr_status mcr_step_sizes_blocks(int32_t n_gates, int32_t n_subsets, const double* norms_sq, double alpha,
                                 double* sigma, double* tau, double* theta, double* rate_per_epoch) {
  if (n_gates < 1) return fail(MCR_ERR_ARG, "n_gates = %d must be >= 1", n_gates);
  if (n_subsets < 1) return fail(MCR_ERR_ARG, "n_subsets = %d must be >= 1", n_subsets);
  STATUS_OK(check_ptr(norms_sq, "norms_sq"));
  STATUS_OK(check_ptr(sigma, "sigma"));
  if (!(alpha > 0) || !std::isfinite(alpha)) return fail(MCR_ERR_ARG, "alpha must be finite and > 0");
  const int nb = n_gates * n_subsets;
  for (int b = 0; b < nb; ++b)
    if (!(norms_sq[b] > 0) || !std::isfinite(norms_sq[b]))
      return fail(MCR_ERR_ARG, "norms_sq[%d] = %g must be finite and > 0", b, norms_sq[b]);
  const double N = n_gates, pr = 1.0 / nb;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double sb = std::sqrt(1.0 + norms_sq[b] / (alpha * N));
    s = std::max(s, sb);
    sigma[b] = 2.0 / (N * (sb - 1.0));
  }
  const double rho = 1.0 - 2.0 * pr / (1.0 + s);
  if (tau) *tau = pr / (2.0 * alpha * rho * (1.0 + s));
  if (theta) *theta = rho;
  if (rate_per_epoch) *rate_per_epoch = std::pow(rho, nb);
  return MCR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Joseph projection that allocates nothing (mcr_project_noalloc).
//
// Its scratch (the per-angle fixed-point table, an identity motion entry and
// the zero-bordered image with its transpose) lives in one file-scope device
// array. Host code never passes the array's name to a kernel: the name is a
// host-side stand-in, so each device's address is looked up once with
// hipGetSymbolAddress (with that device current) and kept per device.
// ---------------------------------------------------------------------------
namespace {

constexpr int kNoallocMaxN = 1024;
constexpr int kNoallocMaxAngles = 4096;
constexpr int kNoallocMaxDevices = 64;
constexpr size_t kNoallocAlign = 256;

constexpr size_t align_up(size_t v) { return (v + kNoallocAlign - 1) / kNoallocAlign * kNoallocAlign; }
constexpr size_t kNoallocAngBytes = align_up(sizeof(AngleFx) * kNoallocMaxAngles);
constexpr size_t kNoallocMotionBytes = align_up(sizeof(GateMotion<float>));
constexpr size_t kNoallocPlaneBytes =
    align_up(sizeof(float) * (size_t)(kNoallocMaxN + 2 * kPad) * (kNoallocMaxN + 2 * kPad));
constexpr size_t kNoallocScratchBytes = kNoallocAngBytes + kNoallocMotionBytes + 2 * kNoallocPlaneBytes;

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[kNoallocMaxDevices] = {};

// The fixed-point table of angle_table_fx, evaluated on the device in FP64
// with the same formulas (contraction off, as in the host code), plus the
// identity motion entry and the zero border of both padded planes. The border
// has to be cleared on every call: the array keeps what earlier calls, maybe
// with another size, wrote there.
#pragma clang fp contract(off)
__global__ __launch_bounds__(256) void k_noalloc_prepare(int n, int na, int nd, AngleFx* __restrict__ ang,
                                                         GateMotion<float>* __restrict__ motion,
                                                         float* __restrict__ wP, float* __restrict__ wTP) {
  const long tid = (long)blockIdx.x * 256 + threadIdx.x;
  const long stride = (long)gridDim.x * 256;
  if (tid < na) {
    const int k = (int)tid;
    const double hc = (n - 1) / 2.0, jc = (nd - 1) / 2.0, one = 4294967296.0;
    const double th = M_PI * k / na;
    const double cs = cos(th), sn = sin(th);
    const bool rows = (4L * k <= na) || (4L * k >= 3L * na);
    const double a = rows ? 1.0 / cs : 1.0 / sn;
    const double beta = rows ? -sn / cs : -cs / sn;
    const double c0 = hc - jc * a - hc * beta;
    const double ia = 1.0 / a;
    AngleFx f;
    f.C0 = llround(c0 * one);
    f.A = llround(a * one);
    f.B = llround(beta * one);
    f.U0 = llround(-c0 * ia * one);
    f.P = llround(ia * one);
    f.Q = llround(-beta * ia * one);
    f.RS = rows ? f.P : f.Q;
    f.a = float(a);
    f.beta = float(beta);
    f.absa = float(fabs(a));
    f.oma = float(1.0 - fabs(a));
    f.ds = float(fabs(a));
    f.rows = rows ? 1 : 0;
    f.na32 = float(-fabs(a) / one);
    f.pa32 = float(fabs(a) / one);
    ang[k] = f;
  }
  if (tid == 0) {
    GateMotion<float> m;
    m.kind = 0;
    m.radius = 0;
    m.cm1 = m.sn = m.tx = m.ty = 0.0f;
    m.i00 = m.i01 = m.i10 = m.i11 = 0.0f;
    m.bx = m.by = 0.0f;
    *motion = m;
  }
  const int pitch = n + 2 * kPad;
  const long cells = (long)pitch * pitch;
  for (long i = tid; i < cells; i += stride) {
    const int r = (int)(i / pitch), c = (int)(i % pitch);
    const bool interior = r >= kPad && r < kPad + n && c >= kPad && c < kPad + n;
    if (!interior) {
      wP[i] = 0.0f;
      wTP[i] = 0.0f;
    }
  }
}
#pragma clang fp contract(on)

// This device's address of `scratch`, looked up on the first call made with
// the device current.
mcr_status noalloc_scratch(unsigned char** out) {
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoallocMaxDevices)
    return fail(MCR_ERR_STATE, "device %d is beyond the %d devices this entry point serves", dev,
                kNoallocMaxDevices);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MCR_ERR_HIP, "hipGetSymbolAddress returned a null address for the scratch array");
    g_noalloc_ptr[dev] = (unsigned char*)p;
  }
  *out = g_noalloc_ptr[dev];
  return MCR_OK;
}

}  // namespace

extern "C" {

mcr_status mcr_project_noalloc(const mcr_geometry* geom, const float* x, float* sino, void* stream) {
  if (!geom) return fail(MCR_ERR_ARG, "null geometry");
  const int n = geom->n, na = geom->n_angles, nd = geom->n_det;
  if (n < 1 || n > kNoallocMaxN)
    return fail(MCR_ERR_ARG, "n = %d outside [1, %d], the largest image this entry point's scratch holds", n,
                kNoallocMaxN);
  if (na < 1 || na > kNoallocMaxAngles)
    return fail(MCR_ERR_ARG, "n_angles = %d outside [1, %d], the largest angle table this entry point's scratch holds",
                na, kNoallocMaxAngles);
  if (nd < 1 || nd > 16384) return fail(MCR_ERR_ARG, "n_det = %d outside [1, 16384]", nd);
  STATUS_OK(check_ptr(x, "x"));
  STATUS_OK(check_ptr(sino, "sino"));
  unsigned char* base = nullptr;
  STATUS_OK(noalloc_scratch(&base));
  AngleFx* ang = (AngleFx*)base;
  GateMotion<float>* motion = (GateMotion<float>*)(base + kNoallocAngBytes);
  float* wP = (float*)(base + kNoallocAngBytes + kNoallocMotionBytes);
  float* wTP = (float*)(base + kNoallocAngBytes + kNoallocMotionBytes + kNoallocPlaneBytes);
  hipStream_t s = (hipStream_t)stream;
  const int pitch = n + 2 * kPad;
  Geo<float> g{n, na, nd, pitch, float((n - 1) / 2.0), float((nd - 1) / 2.0)};
  hipLaunchKernelGGL(k_noalloc_prepare, dim3(std::max<unsigned>(cdiv(na, 256), cdiv((long)pitch * pitch, 1024))),
                     dim3(256), 0, s, n, na, nd, ang, motion, wP, wTP);
  LAUNCH_OK();
  // the identity warp copies x into both padded planes (row-major and
  // transposed); it never reads the field argument of an identity gate
  hipLaunchKernelGGL(k_warp_fwd<float>, dim3(cdiv(n, 32), cdiv(n, 32), 1), dim3(32, 32), 0, s, g,
                     (const GateMotion<float>*)motion, 0, (const float*)wP, 0L, 0L, x, 0L, wP, wTP, 0L,
                     (const SlotInfo*)nullptr, (float*)nullptr, 0L, 0L, 0);
  LAUNCH_OK();
  hipLaunchKernelGGL((k_joseph_fwd_fx<0>), dim3(cdiv(nd, 256), na, 1), dim3(256), 0, s, g,
                     (const AngleFx*)ang, (const float*)wP, (const float*)wTP, 0L, sino, 0L, 0,
                     (const GateScalars<float>*)nullptr, (const GatePtrs<float>*)nullptr, (const SlotInfo*)nullptr, 0);
  LAUNCH_OK();
  return MCR_OK;
}

}  // extern "C"
