// C ABI of libdycore: handle life cycle, step sequencing, diagnostics, batches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/dycore.h"
#include "dycore_internal.h"

using namespace dyc;

namespace {

constexpr int kPoleSlots = 8;

// Row partials of dycore_diagnostics_noalloc: a file-scope device array, one copy per GPU, held
// until the process ends.  Host code never passes its name to a kernel (on the host it stands for
// no device address); it uses the address hipGetSymbolAddress returns for each device.
constexpr int kNoallocMaxRows = 4097;                  // ny + 1 <= 4097 (0.044-degree rows)
constexpr int kNoallocDoubles = 3 * kNoallocMaxRows + 2;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[kNoallocDoubles];

namespace {

// Resolves, once per device and with that device current, the address of `scratch` on it.
int resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return DYCORE_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return DYCORE_OK;
  double* ptr = nullptr;
  if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DYCORE_EHIP;
  g_scratch_dev[device] = ptr;
  return DYCORE_OK;
}

struct DeviceBuf {
  void* p = nullptr;
  size_t n = 0;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

struct dycore_s {
  int nx, ny, nz, prec, msub, block;
  unsigned flags;
  double dt;
  int device;
  GeoDev g;
  GeoFac fac;
  int recorded = 0;             // the adjoint workspace holds the stage inputs of a recorded step
  dyc::KTimer timer;            // live timing of the row-fused adaptation-stage adjoint
  std::vector<int> M, Mv;
  size_t nU, nV, nF, nP;        // element counts of each field
  size_t elem;                  // 4 or 8
  size_t state_bytes;           // bytes of one packed state (U|V|F|P, 256-aligned parts)
  void* geo = nullptr;          // tables
  void* scratch = nullptr;      // forward scratch: y1, y2
  double* pole = nullptr;       // kPoleSlots x 2 x (nz+1)
  double* diag = nullptr;       // 3*(ny+1) row partials, then the 2 global sums
  unsigned long long* count = nullptr;
  void* adj = nullptr;          // adjoint workspace
  size_t adj_bytes = 0;
  AatItem* aat = nullptr;       // work items of the tiled adaptation-stage adjoint (device)
  int aat_n = 0, aat_block = 0, aat_edge_n = 0;   // aat_edge_n: rows 1 and ny-1 after the others
  AatItem* adt = nullptr;       // work items of the tiled advection-stage adjoint (device)
  int adt_n = 0, adt_block = 0;
  int adt_pp_n = 0, adt_pp_s = 0;   // interior rows at each end that run the per-point kernels
  FiltItem* filt = nullptr;     // rows of the low-latitude filters (device), when enabled
  int nfilt = 0;
  AatItem* ftiles = nullptr;    // zonal tiles of the forward adaptation stage (device), rows 0..ny
  int nftiles = 0, ftblock = 0;
  AatItem* atiles = nullptr;    // zonal tiles of the forward advection stage (device): the main
  int natiles = 0, awide = 0;   // launch's (workgroups of `block` threads; awide: it has wide tiles),
  int nptiles = 0, pblock = 0;  // then the polar launch's (wide tiles) at atiles + natiles
  dyc::SideLaunch side{nullptr, nullptr, nullptr};   // second stream and events: band beside polar tiles
  double* cap = nullptr;        // cap sums of the forward adaptation stage: [2 poles][2][nz]
  size_t bytes = 0;
};

size_t dyc_adjoint_workspace_bytes(const dycore_s* h);

struct dycore_batch_s {
  int n, prec, block, grid, max_nx, nstage_max;
  size_t lds;   // dynamic LDS of the batched stage kernel: the largest need of any member
  std::vector<dycore_t> hs;
  void* d_args = nullptr;       // nstage_max x n StageArgs
  int2* d_items = nullptr;      // advection tiles (member, index into the member's advection tile table)
  int nitems = 0;
  int2* d_titems = nullptr;     // adaptation tiles (member, index into the member's tile table)
  int ntitems = 0;
  AatItem* d_tiles = nullptr;   // every member's adaptation and advection tile tables for the batch's block
  int max_nz = 0;
  void* d_prep = nullptr;       // per member prep descriptors
  std::vector<void*> U, V, F, P;
};

namespace {

template <typename T>
struct Packed {
  T* U; T* V; T* F; T* P;
};

template <typename T>
Packed<T> unpack(const dycore_s* h, void* base) {
  char* c = static_cast<char*>(base);
  Packed<T> s;
  s.U = reinterpret_cast<T*>(c);
  c += align256(h->nU * sizeof(T));
  s.V = reinterpret_cast<T*>(c);
  c += align256(h->nV * sizeof(T));
  s.F = reinterpret_cast<T*>(c);
  c += align256(h->nF * sizeof(T));
  s.P = reinterpret_cast<T*>(c);
  return s;
}

double* pole_slot(const dycore_s* h, int s) { return h->pole + (size_t)s * 2 * (h->nz + 1); }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int hip_status(hipError_t e) { return e == hipSuccess ? DYCORE_OK : DYCORE_EHIP; }

int leap_span(double sin_theta, double dlam, int nx) {
  // eq. 7 with res = dlam, cos(90 deg - theta) = sin(theta); ceiling, then odd (Sec. III-B), then < nx/2
  const double r = std::asin(std::cos(M_PI / 4.0) * std::sin(dlam)) / std::asin(sin_theta * std::sin(dlam));
  int m = (int)std::ceil(r - 1e-9);
  if (m < 1) m = 1;
  if ((m & 1) == 0) ++m;
  int cap = (nx - 1) / 2;
  if ((cap & 1) == 0) --cap;
  if (cap < 1) cap = 1;
  return std::min(m, cap);
}

// Rows the low-latitude filters act on (Sec. III-B, Table IV rows 1-2).  The latitude of scalar
// and U row j is 90 (ny - 2j) / ny degrees, of V row j 90 (ny - 2j - 1) / ny; the band edges are
// decided on those integers: below 38 degrees the simplified filter (r = -1), from 38 to 70 the
// 3-point operator with r = (1 - cos(lat) / cos 38deg) / 4 (rows where it vanishes are skipped),
// poleward of 70 nothing.
std::vector<FiltItem> filter_items(int ny) {
  auto coef = [&](int num) {
    const int m = num < 0 ? -num : num;
    if (m * 90 < 38 * ny) return -1.0;
    if (m * 90 > 70 * ny) return 0.0;
    const double lat = 90.0 * m / ny * (M_PI / 180.0);
    return 0.25 * (1.0 - std::cos(lat) / std::cos(38.0 * M_PI / 180.0));
  };
  std::vector<FiltItem> out;
  for (int j = 1; j < ny; ++j) {
    const double r = coef(ny - 2 * j);
    if (r == 0.0) continue;
    out.push_back(FiltItem{0, j, r});
    out.push_back(FiltItem{2, j, r});
    out.push_back(FiltItem{3, j, r});
  }
  for (int j = 0; j < ny; ++j) {
    const double r = coef(ny - 2 * j - 1);
    if (r != 0.0) out.push_back(FiltItem{1, j, r});
  }
  return out;
}

// Zonal tiles of the listed rows for a block of `block` threads: every row is cut into the fewest
// equal tiles whose owned columns plus a halo of hl[j] columns on each side fit the block.  Items are
// listed row by row, then spread so that item b (which the hardware dispatches to XCD b mod 8) walks
// a contiguous eighth of that list.  Returns false when some row's halo leaves fewer than 32 owned
// columns.
bool zonal_tiles(int nx, const std::vector<int>& rows, const std::vector<int>& hl, int block,
                 std::vector<AatItem>& out) {
  std::vector<AatItem> seq;
  for (const int j : rows) {
    const int cap = block - 2 * hl[j];
    if (cap < 32) return false;
    const int nt = (nx + cap - 1) / cap;
    const int w = (nx + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
      const int i0 = t * w;
      if (i0 >= nx) break;
      seq.push_back(AatItem{j, i0, std::min(w, nx - i0), hl[j]});
    }
  }
  const int n = (int)seq.size(), per = (n + 7) / 8;
  out.assign((size_t)per * 8, AatItem{-1, 0, 0, 0});
  for (int x = 0; x < 8; ++x)
    for (int q = 0; q < per; ++q) {
      const int src = x * per + q;
      if (src < n) out[(size_t)q * 8 + x] = seq[src];
    }
  return true;
}

// The block (a multiple of 64 up to max_block) whose tiles of the listed rows leave the fewest idle
// threads (owned columns over launched threads; ties go to the larger block), and its items.  False
// when no block fits the widest halo.
bool best_tiles(int nx, const std::vector<int>& rows, const std::vector<int>& hl, int max_block,
                std::vector<AatItem>& out, int& block) {
  double best = -1.0;
  for (int b = 64; b <= max_block; b += 64) {
    std::vector<AatItem> items;
    if (!zonal_tiles(nx, rows, hl, b, items)) continue;
    const double util = (double)nx * rows.size() / ((double)items.size() * b);
    if (util >= best - 1e-12) {
      best = util;
      block = b;
      out.swap(items);
    }
  }
  return best > 0.0;
}

// Rows j0..j1 (j1 < 0: ny - 1) and the halo n_j + 1 of the adaptation stage and its adjoint, whose
// leaped differences reach n_j columns and whose U-V averages one more.
std::vector<int> row_range(int j0, int j1) {
  std::vector<int> r;
  for (int j = j0; j <= j1; ++j) r.push_back(j);
  return r;
}
std::vector<int> adapt_halos(const std::vector<int>& M) {
  std::vector<int> hl(M.size());
  for (size_t j = 0; j < M.size(); ++j) hl[j] = (M[j] + 1) / 2 + 1;
  return hl;
}

// Work items of the tiled adaptation stage and its adjoint for a block of `block` threads.
bool aat_tiles(int nx, int ny, const std::vector<int>& M, int block, std::vector<AatItem>& out, int j0 = 1,
               int j1 = -1) {
  return zonal_tiles(nx, row_range(j0, j1 < 0 ? ny - 1 : j1), adapt_halos(M), block, out);
}

// The best block up to max_block for those tiles (false when no block fits the widest halo: the
// adjoint then uses its per-point kernels).
bool aat_items(int nx, int ny, const std::vector<int>& M, std::vector<AatItem>& out, int& block, int j0 = 1,
               int j1 = -1, int max_block = kAatMaxBlock) {
  return best_tiles(nx, row_range(j0, j1 < 0 ? ny - 1 : j1), adapt_halos(M), max_block, out, block);
}

// Work items of the tiled advection-stage adjoint.  Its centred leaped differences span 2 M, so a
// row's halo is the largest leap of the row and its V rows: max(M_j, Mv_j, nv_{j-1}).  Rows whose
// halo leaves 32 owned columns in 256 threads are tiled; the others must be the first pp_n and the
// last pp_s interior rows (next to the poles, where the leaps grow), which run the per-point
// kernels with the pole rows.  False when no row is tiled or the others are not at the ends.
bool adt_items(int nx, int ny, const std::vector<int>& M, const std::vector<int>& Mv, std::vector<AatItem>& out,
               int& block, int& pp_n, int& pp_s) {
  std::vector<int> hl(ny + 1, 0), rows;
  std::vector<char> fits(ny + 1, 0);
  for (int j = 1; j <= ny - 1; ++j) {
    hl[j] = std::max(std::max(M[j], Mv[j]), (Mv[j - 1] + 1) / 2);
    fits[j] = 256 - 2 * hl[j] >= 32;
    if (fits[j]) rows.push_back(j);
  }
  out.clear();
  block = pp_n = pp_s = 0;
  if (rows.empty()) return false;
  pp_n = rows.front() - 1;
  pp_s = ny - 1 - rows.back();
  if ((int)rows.size() != rows.back() - rows.front() + 1) return false;
  return best_tiles(nx, rows, hl, 256, out, block);
}

// Work items of the tiled advection stage of one member, for a main launch and a polar launch, both
// of `block` threads: a row takes band tiles in the main launch when its halo (as below) leaves 32
// owned columns, else wide tiles (halo 1, leap operands from global memory) in the polar launch,
// which runs beside the main one.  Both lists are XCD-spread as zonal_tiles.
void advect_tiles_split(int nx, int ny, const std::vector<int>& M, const std::vector<int>& Mv, int block,
                        std::vector<AatItem>& main, std::vector<AatItem>& polar) {
  std::vector<AatItem> wide, band, pol;
  auto cut = [&](int j, int hl, int cap, int hmark, std::vector<AatItem>& to) {
    const int nt = (nx + cap - 1) / cap;
    const int w = (nx + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
      const int i0 = t * w;
      if (i0 >= nx) break;
      to.push_back(AatItem{j, i0, std::min(w, nx - i0), hmark});
    }
    (void)hl;
  };
  for (int j = 0; j <= ny; ++j) {
    const int hl = std::max((j == 0 || j == ny) ? 1 : M[j], j < ny ? Mv[j] : 1);
    if (block - 2 * hl >= 32) cut(j, hl, block - 2 * hl, hl, band);
    else cut(j, hl, block - 2, -1, pol);
  }
  auto spread = [](const std::vector<AatItem>& seq, std::vector<AatItem>& out) {
    const int n = (int)seq.size(), per = (n + 7) / 8;
    out.assign((size_t)per * 8, AatItem{-1, 0, 0, 0});
    for (int x = 0; x < 8; ++x)
      for (int q = 0; q < per; ++q) {
        const int src = x * per + q;
        if (src < n) out[(size_t)q * 8 + x] = seq[src];
      }
  };
  (void)wide;
  spread(band, main);
  polar.clear();
  if (!pol.empty()) spread(pol, polar);
}

// Work items of the tiled advection stage for a block of `block` threads (rows 0..ny).  A row's halo
// is the reach of its leaped centred differences, max(M_j, Mv_j, 1) (the pole rows have no zonal
// Phi and U terms); rows whose halo leaves 32 owned columns take band tiles, the others wide tiles
// (a halo of one column, hl = -1 in the item) that read their leap operands from global memory.
// Wide items lead the list, so that they start first.
void advect_tiles(int nx, int ny, const std::vector<int>& M, const std::vector<int>& Mv, int block,
                  std::vector<AatItem>& out) {
  std::vector<AatItem> wide, band;
  for (int j = 0; j <= ny; ++j) {
    const int hl = std::max((j == 0 || j == ny) ? 1 : M[j], j < ny ? Mv[j] : 1);
    const bool fits = block - 2 * hl >= 32;
    const int cap = fits ? block - 2 * hl : block - 2;
    const int nt = (nx + cap - 1) / cap;
    const int w = (nx + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
      const int i0 = t * w;
      if (i0 >= nx) break;
      (fits ? band : wide).push_back(AatItem{j, i0, std::min(w, nx - i0), fits ? hl : -1});
    }
  }
  std::vector<AatItem> seq(wide);
  seq.insert(seq.end(), band.begin(), band.end());
  const int n = (int)seq.size(), per = (n + 7) / 8;
  out.assign((size_t)per * 8, AatItem{-1, 0, 0, 0});
  for (int x = 0; x < 8; ++x)
    for (int q = 0; q < per; ++q) {
      const int src = x * per + q;
      if (src < n) out[(size_t)q * 8 + x] = seq[src];
    }
}

// The polar advection tiles' stream of a handle (NULL when it has none).
const dyc::SideLaunch* side_of(const dycore_s* h) { return h->side.s ? &h->side : nullptr; }

template <typename T>
StageArgs<T> make_args(const dycore_s* h, int process, double ch, const T* inU, const T* inV, const T* inF,
                       const T* inP, const T* bU, const T* bV, const T* bF, const T* bP, T* oU, T* oV, T* oF,
                       T* oP, const double* pin, const double* pbase, double* pout) {
  StageArgs<T> a;
  a.g = h->g;
  a.inU = inU; a.inV = inV; a.inF = inF; a.inP = inP;
  a.bU = bU; a.bV = bV; a.bF = bF; a.bP = bP;
  a.oU = oU; a.oV = oV; a.oF = oF; a.oP = oP;
  a.pin = pin; a.pbase = pbase; a.pout = pout;
  a.ch = ch;
  a.process = process;
  a.pad = 0;
  a.tiles = h->ftiles;
  a.cap = h->cap;
  a.ntiles = h->nftiles;
  a.tblock = h->ftblock;
  a.atiles = h->atiles;
  a.natiles = h->natiles;
  a.ablock = h->block;
  a.awide = h->awide;
  a.ptiles = h->nptiles > 0 ? h->atiles + h->natiles : nullptr;
  a.nptiles = h->nptiles;
  a.pblock = h->pblock;
  return a;
}

// Pole-value slots of one outer step.  Slot 0 holds the pole values of the
// step's start state and is written only by the last stage of the step, so the
// next step (or the next replay of a batch) finds its start values there.  RK
// step rk has base slot b; its stages write s1 (y1), s2 (y2) and then the next
// base, which reuses s1.
struct Slots { int pin, pbase, pout; };

Slots stage_slots(int rk, int nrk, int r) {
  int b = 0;
  for (int q = 0; q < rk; ++q) b = (b == 0) ? 1 : (b % 3) + 1;
  const int s1 = (b == 0) ? 1 : (b % 3) + 1;
  const int s2 = (s1 % 3) + 1;
  if (r == 0) return {b, b, s1};
  if (r == 1) return {s1, b, s2};
  return {s2, b, (rk == nrk - 1) ? 0 : s1};
}

// Arguments of stage r (0..2) of RK step rk of one outer step: y1 = y + h/3 T(y),
// y2 = y + h/2 T(y1), y <- y + h T(y2), with T the adaptation for the first msub
// RK steps (h = dt/msub) and the advection for the last (h = dt).
template <typename T>
StageArgs<T> step_stage_args(const dycore_s* h, int rk, int r, T* U, T* V, T* F, T* P) {
  Packed<T> y1 = unpack<T>(h, h->scratch);
  Packed<T> y2 = unpack<T>(h, static_cast<char*>(h->scratch) + h->state_bytes);
  const int nrk = h->msub + 1;
  const int proc = (rk < h->msub) ? 0 : 1;
  const double hs = proc == 0 ? h->dt / h->msub : h->dt;
  const Slots sl = stage_slots(rk, nrk, r);
  const double* pin = pole_slot(h, sl.pin);
  const double* pb = pole_slot(h, sl.pbase);
  double* po = pole_slot(h, sl.pout);
  if (r == 0)
    return make_args<T>(h, proc, hs / 3.0, U, V, F, P, U, V, F, P, y1.U, y1.V, y1.F, y1.P, pin, pb, po);
  if (r == 1)
    return make_args<T>(h, proc, hs / 2.0, y1.U, y1.V, y1.F, y1.P, U, V, F, P, y2.U, y2.V, y2.F, y2.P, pin, pb, po);
  return make_args<T>(h, proc, hs, y2.U, y2.V, y2.F, y2.P, U, V, F, P, U, V, F, P, pin, pb, po);
}

template <typename T>
int step_impl(dycore_s* h, T* U, T* V, T* F, T* P, int nsteps, hipStream_t s) {
  if (nsteps == 0) return DYCORE_OK;
  hipError_t e = launch_pole_prep<T>(h->g, F, P, pole_slot(h, 0), s);
  if (e != hipSuccess) return DYCORE_EHIP;
  const int nrk = h->msub + 1;
  for (int n = 0; n < nsteps; ++n) {
    for (int rk = 0; rk < nrk; ++rk)
      for (int r = 0; r < 3; ++r) {
        e = launch_stage<T>(step_stage_args<T>(h, rk, r, U, V, F, P), s, side_of(h));
        if (e != hipSuccess) return DYCORE_EHIP;
      }
    // the low-latitude filters close the step (they leave the pole rows and their slot alone)
    e = launch_lowlat<T>(h->g, h->filt, h->nfilt, U, V, F, P, s);
    if (e != hipSuccess) return DYCORE_EHIP;
  }
  return DYCORE_OK;
}

// n_rk RK3 steps of one process with step hstep (the 3 stage launches of each
// exactly as in an outer step, pole slots 0 -> ... -> 0).
template <typename T>
int process_run_impl(dycore_s* h, int process, int n_rk, double hstep, T* U, T* V, T* F, T* P, hipStream_t s) {
  if (n_rk == 0) return DYCORE_OK;
  hipError_t e = launch_pole_prep<T>(h->g, F, P, pole_slot(h, 0), s);
  if (e != hipSuccess) return DYCORE_EHIP;
  Packed<T> y1 = unpack<T>(h, h->scratch);
  Packed<T> y2 = unpack<T>(h, static_cast<char*>(h->scratch) + h->state_bytes);
  int b = 0;   // base pole slot alternates between 0 and 3
  for (int n = 0; n < n_rk; ++n) {
    const int nb = (b == 0) ? 3 : 0;
    e = launch_stage<T>(make_args<T>(h, process, hstep / 3.0, U, V, F, P, U, V, F, P, y1.U, y1.V, y1.F, y1.P,
                                     pole_slot(h, b), pole_slot(h, b), pole_slot(h, 1)), s, side_of(h));
    if (e == hipSuccess)
      e = launch_stage<T>(make_args<T>(h, process, hstep / 2.0, y1.U, y1.V, y1.F, y1.P, U, V, F, P, y2.U, y2.V,
                                       y2.F, y2.P, pole_slot(h, 1), pole_slot(h, b), pole_slot(h, 2)), s, side_of(h));
    if (e == hipSuccess)
      e = launch_stage<T>(make_args<T>(h, process, hstep, y2.U, y2.V, y2.F, y2.P, U, V, F, P, U, V, F, P,
                                       pole_slot(h, 2), pole_slot(h, b), pole_slot(h, nb)), s, side_of(h));
    if (e != hipSuccess) return DYCORE_EHIP;
    b = nb;
  }
  return DYCORE_OK;
}

template <typename T>
int stage_impl(dycore_s* h, int process, double ch, const T* bU, const T* bV, const T* bF, const T* bP,
               const T* U, const T* V, const T* F, const T* P, T* oU, T* oV, T* oF, T* oP, hipStream_t s) {
  hipError_t e = launch_pole_prep<T>(h->g, F, P, pole_slot(h, 0), s);
  if (e == hipSuccess) e = launch_pole_prep<T>(h->g, bF, bP, pole_slot(h, 1), s);
  if (e == hipSuccess)
    e = launch_stage<T>(make_args<T>(h, process, ch, U, V, F, P, bU, bV, bF, bP, oU, oV, oF, oP, pole_slot(h, 0),
                                     pole_slot(h, 1), pole_slot(h, 2)), s, side_of(h));
  return hip_status(e);
}

void release_timer(dycore_s* h) {
  dyc::KTimer& t = h->timer;
  if (t.ev) {
    for (int q = 0; q < 2 * t.cap; ++q) (void)hipEventDestroy(t.ev[q]);
    delete[] t.ev;
  }
  t = dyc::KTimer{};
}

// Fewest adaptation sub-steps that keep dt / M within the CFL bound of the fastest gravity wave
// on the 45-degree reference spacing (eq. 6's reference row): ceil(w_max dt / (0.8 sqrt 3)) with
// w_max = 2 c sqrt(1/dx45^2 + 1/dy^2), c = 350 m/s.
int cfl_substeps(const dycore_config* c) {
  const double a = c->a != 0.0 ? c->a : 6.371e6;
  const double dx45 = a * std::cos(M_PI / 4.0) * (2.0 * M_PI / c->nx), dy = a * (M_PI / c->ny);
  const double wmax = 2.0 * 350.0 * std::sqrt(1.0 / (dx45 * dx45) + 1.0 / (dy * dy));
  return std::max(1, (int)std::ceil(wmax * c->dt / (0.8 * std::sqrt(3.0))));
}

int validate_cfg(const dycore_config* c) {
  if (!c) return DYCORE_EINVAL;
  if (c->nx < 8 || c->nx > 4096 || c->ny < 4 || c->ny > 8192 || c->nz < 1 || c->nz > kMaxLevels) return DYCORE_EINVAL;
  if (!(c->dt > 0.0) || !std::isfinite(c->dt)) return DYCORE_EINVAL;
  if (c->n_adapt_substeps < 0) return DYCORE_EINVAL;
  if (c->prec != DYCORE_FP32 && c->prec != DYCORE_FP64) return DYCORE_EINVAL;
  if (c->block != 0 && (c->block < 64 || c->block > 1024 || (c->block % 64) != 0)) return DYCORE_EINVAL;
  // kernels address a field's rows with 32-bit byte offsets: every field (half levels included)
  // stays below 4 GiB
  const size_t elem = c->prec == DYCORE_FP64 ? 8 : 4;
  if ((size_t)c->nx * (size_t)(c->ny + 1) * (size_t)(c->nz + 1) * elem >= (size_t(1) << 32)) return DYCORE_EINVAL;
  // a given sub-step count must keep the adaptation sub-step within the CFL bound of the
  // gravity-wave speed: w_max dt / M <= 0.8 sqrt 3 (the count chosen when M = 0)
  if (c->n_adapt_substeps > 0 && cfl_substeps(c) > c->n_adapt_substeps) return DYCORE_EINVAL;
  // the simplified filter removes the 2-dlam wave, which needs an even number of columns
  if ((c->flags & DYCORE_LOWLAT_FILTERS) && (c->nx % 2) != 0) return DYCORE_EINVAL;
  if (!(c->kappa_star >= 0.0) || !std::isfinite(c->kappa_star)) return DYCORE_EINVAL;
  if (c->sigma_half) {
    if (c->sigma_half[0] != 0.0 || c->sigma_half[c->nz] != 1.0) return DYCORE_EINVAL;
    for (int k = 0; k < c->nz; ++k)
      if (!(c->sigma_half[k + 1] > c->sigma_half[k])) return DYCORE_EINVAL;
  }
  return DYCORE_OK;
}

}  // namespace

dyc::HandleView dyc::view_of(const dycore_s* h) {
  HandleView v;
  v.g = h->g;
  v.prec = h->prec;
  v.msub = h->msub;
  v.dt = h->dt;
  v.nU = h->nU; v.nV = h->nV; v.nF = h->nF; v.nP = h->nP;
  v.elem = h->elem;
  v.state_bytes = h->state_bytes;
  v.adj = h->adj;
  v.adj_bytes = h->adj_bytes;
  v.pole = h->pole;
  v.scratch = h->scratch;
  v.block = h->block;
  v.fac = h->fac;
  v.recorded = const_cast<int*>(&h->recorded);
  v.timer = const_cast<dyc::KTimer*>(&h->timer);
  v.aat = h->aat;
  v.aat_n = h->aat_n;
  v.aat_block = h->aat_block;
  v.aat_edge_n = h->aat_edge_n;
  v.adt = h->adt;
  v.adt_n = h->adt_n;
  v.adt_block = h->adt_block;
  v.adt_pp_n = h->adt_pp_n;
  v.adt_pp_s = h->adt_pp_s;
  v.filt = h->filt;
  v.nfilt = h->nfilt;
  v.ftiles = h->ftiles;
  v.nftiles = h->nftiles;
  v.ftblock = h->ftblock;
  v.atiles = h->atiles;
  v.natiles = h->natiles;
  v.ablock = h->block;
  v.awide = h->awide;
  v.ptiles = h->nptiles > 0 ? h->atiles + h->natiles : nullptr;
  v.nptiles = h->nptiles;
  v.pblock = h->pblock;
  v.side = h->side.s ? &h->side : nullptr;
  v.adj_side = h->side.s && !(h->flags & DYCORE_FORWARD_ONLY) &&
                       (size_t)h->nx * h->ny * h->nz >= kAdjOverlapPoints ? &h->side : nullptr;
  v.cap = h->cap;
  return v;
}

extern "C" {

const char* dycore_strerror(int status) {
  switch (status) {
    case DYCORE_OK: return "ok";
    case DYCORE_EINVAL: return "invalid argument";
    case DYCORE_ENOMEM: return "device allocation failed";
    case DYCORE_EHIP: return "HIP runtime error";
    case DYCORE_ENONFINITE: return "non-finite value in a field";
    case DYCORE_EUNSUPPORTED: return "grid exceeds a kernel tile limit";
    default: return "unknown status";
  }
}

int dycore_create(const dycore_config* cfg, dycore_t* out) {
  if (!out) return DYCORE_EINVAL;
  *out = nullptr;
  int st = validate_cfg(cfg);
  if (st != DYCORE_OK) return st;
  dycore_s* h = new (std::nothrow) dycore_s();
  if (!h) return DYCORE_ENOMEM;
  h->nx = cfg->nx; h->ny = cfg->ny; h->nz = cfg->nz; h->prec = cfg->prec; h->dt = cfg->dt; h->flags = cfg->flags;
  h->elem = (h->prec == DYCORE_FP32) ? 4 : 8;
  // the tiled advection stage's workgroup (its kernel's register budget is set for 256 threads)
  h->block = cfg->block ? std::min(cfg->block, 256) : 256;
  (void)hipGetDevice(&h->device);
  if ((st = resolve_scratch(h->device)) != DYCORE_OK) { delete h; return st; }

  const int nx = h->nx, ny = h->ny, nz = h->nz;
  GeoDev& g = h->g;
  g.nx = nx; g.ny = ny; g.nz = nz;
  const double defs[7] = {6.371e6, 7.292e-5, 9.80616, 287.04, 1004.64, 1.0e5, 300.0};
  const double given[7] = {cfg->a, cfg->omega, cfg->g, cfg->rd, cfg->cp, cfg->p0, cfg->t0};
  double cst[7];
  for (int i = 0; i < 7; ++i) cst[i] = given[i] != 0.0 ? given[i] : defs[i];
  g.a = cst[0]; g.omega = cst[1]; g.g = cst[2]; g.rd = cst[3]; g.cp = cst[4]; g.p0 = cst[5]; g.t0 = cst[6];
  g.kappa = g.rd / g.cp;
  g.b = std::sqrt(g.kappa * g.rd * g.t0);
  g.RT0 = g.rd * g.t0;
  g.dlam = 2.0 * M_PI / nx;
  g.dth = M_PI / ny;
  g.acap = 2.0 * M_PI * g.a * g.a * (1.0 - std::cos(0.5 * g.dth));
  g.kstar = cfg->kappa_star;

  // host tables
  std::vector<double> s(ny + 1, 0.0), cot(ny + 1, 0.0), f(ny + 1, 0.0);
  std::vector<double> sv(ny), cotv(ny), fv(ny);
  h->M.assign(ny + 1, 1);
  h->Mv.assign(ny, 1);
  for (int j = 1; j < ny; ++j) {
    const double th = j * g.dth;
    s[j] = std::sin(th);
    cot[j] = std::cos(th) / std::sin(th);
    f[j] = 2.0 * g.omega * std::cos(th);
    h->M[j] = leap_span(s[j], g.dlam, nx);
  }
  for (int j = 0; j < ny; ++j) {
    const double th = (j + 0.5) * g.dth;
    sv[j] = std::sin(th);
    cotv[j] = std::cos(th) / std::sin(th);
    fv[j] = 2.0 * g.omega * std::cos(th);
    h->Mv[j] = leap_span(sv[j], g.dlam, nx);
  }
  std::vector<double> sigh(nz + 1), sig(nz), dsig(nz), cl(nz), cpk(nz);
  for (int k = 0; k <= nz; ++k) sigh[k] = cfg->sigma_half ? cfg->sigma_half[k] : double(k) / nz;
  for (int k = 0; k < nz; ++k) {
    sig[k] = 0.5 * (sigh[k] + sigh[k + 1]);
    dsig[k] = sigh[k + 1] - sigh[k];
    cl[k] = k >= 1 ? std::log(sigh[k + 1] / sigh[k]) : 0.0;
    cpk[k] = std::log(sigh[k + 1] / sig[k]);
  }
  std::vector<double> phis((size_t)(ny + 1) * nx, 0.0);
  if (cfg->phis) std::memcpy(phis.data(), cfg->phis, sizeof(double) * phis.size());
  for (int p : {0, ny}) {
    double m = 0;
    for (int i = 0; i < nx; ++i) m += phis[(size_t)p * nx + i];
    m /= nx;
    for (int i = 0; i < nx; ++i) phis[(size_t)p * nx + i] = m;
  }
  auto rnd = [&](double x) { return h->prec == DYCORE_FP32 ? (double)(float)x : x; };
  std::vector<double> rdx(ny + 1, 0.0), rdy(ny + 1, 0.0), rdxv2(ny), rdyv2(ny), r2d(nz), rsig(nz);
  for (int j = 1; j < ny; ++j) {
    rdx[j] = rnd(1.0 / ((double)h->M[j] * g.a * s[j] * g.dlam));
    rdy[j] = rnd(1.0 / (g.a * s[j] * g.dth));
  }
  for (int j = 0; j < ny; ++j) {
    rdxv2[j] = rnd(1.0 / (2.0 * (double)h->Mv[j] * g.a * sv[j] * g.dlam));
    rdyv2[j] = rnd(1.0 / (2.0 * g.a * sv[j] * g.dth));
  }
  for (int k = 0; k < nz; ++k) r2d[k] = 1.0 / (2.0 * dsig[k]);
  for (int k = 0; k < nz; ++k) rsig[k] = 1.0 / sig[k];
  h->msub = cfg->n_adapt_substeps > 0 ? cfg->n_adapt_substeps : cfl_substeps(cfg);

  // one device block for the tables
  std::vector<std::pair<const void*, size_t>> parts = {
      {s.data(), s.size() * 8},       {cot.data(), cot.size() * 8},   {f.data(), f.size() * 8},
      {h->M.data(), h->M.size() * 4}, {sv.data(), sv.size() * 8},     {cotv.data(), cotv.size() * 8},
      {fv.data(), fv.size() * 8},     {h->Mv.data(), h->Mv.size() * 4}, {sigh.data(), sigh.size() * 8},
      {sig.data(), sig.size() * 8},   {dsig.data(), dsig.size() * 8}, {cl.data(), cl.size() * 8},
      {cpk.data(), cpk.size() * 8},   {phis.data(), phis.size() * 8}, {rdx.data(), rdx.size() * 8},
      {rdy.data(), rdy.size() * 8},   {rdxv2.data(), rdxv2.size() * 8}, {rdyv2.data(), rdyv2.size() * 8},
      {r2d.data(), r2d.size() * 8},   {rsig.data(), rsig.size() * 8}};
  size_t gbytes = 0;
  for (auto& pr : parts) gbytes += align256(pr.second);
  if (hipMalloc(&h->geo, gbytes) != hipSuccess) { delete h; return DYCORE_ENOMEM; }
  std::vector<char> host(gbytes, 0);
  std::vector<size_t> off;
  size_t o = 0;
  for (auto& pr : parts) {
    std::memcpy(host.data() + o, pr.first, pr.second);
    off.push_back(o);
    o += align256(pr.second);
  }
  if (hipMemcpy(h->geo, host.data(), gbytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(h->geo); delete h; return DYCORE_EHIP;
  }
  char* gb = static_cast<char*>(h->geo);
  g.s = (const double*)(gb + off[0]); g.cot = (const double*)(gb + off[1]); g.f = (const double*)(gb + off[2]);
  g.M = (const int*)(gb + off[3]); g.sv = (const double*)(gb + off[4]); g.cotv = (const double*)(gb + off[5]);
  g.fv = (const double*)(gb + off[6]); g.Mv = (const int*)(gb + off[7]); g.sigh = (const double*)(gb + off[8]);
  g.sig = (const double*)(gb + off[9]); g.dsig = (const double*)(gb + off[10]); g.cl = (const double*)(gb + off[11]);
  g.cpk = (const double*)(gb + off[12]); g.phis = (const double*)(gb + off[13]);
  h->fac.rdx = (const double*)(gb + off[14]); h->fac.rdy = (const double*)(gb + off[15]);
  h->fac.rdxv2 = (const double*)(gb + off[16]); h->fac.rdyv2 = (const double*)(gb + off[17]);
  h->fac.r2d = (const double*)(gb + off[18]);
  h->fac.rsig = (const double*)(gb + off[19]);

  h->nU = (size_t)(ny + 1) * nz * nx;
  h->nV = (size_t)ny * nz * nx;
  h->nF = h->nU;
  h->nP = (size_t)(ny + 1) * nx;
  h->state_bytes = align256(h->nU * h->elem) + align256(h->nV * h->elem) + align256(h->nF * h->elem) +
                   align256(h->nP * h->elem);
  h->bytes = gbytes;
  bool ok = hipMalloc(&h->scratch, 2 * h->state_bytes) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->pole, sizeof(double) * kPoleSlots * 2 * (nz + 1)) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->diag, sizeof(double) * (3 * (ny + 1) + 2)) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->count, sizeof(unsigned long long)) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->cap, sizeof(double) * 4 * nz) == hipSuccess;
  if (ok) {
    // the forward adaptation stage covers every scalar row, the poles (span 1) included
    std::vector<AatItem> ft;
    int fblk = 0;
    // blocks of at most 256 threads leave room for several workgroups per CU; grids whose polar
    // halos need more take up to 1024 threads (FP64: 704, for the LDS)
    const int fmax = h->prec == DYCORE_FP32 ? kFwdTileMaxBlock : 704;
    if (!aat_items(nx, ny, h->M, ft, fblk, 0, ny, 256) && !aat_items(nx, ny, h->M, ft, fblk, 0, ny, fmax)) {
      dycore_destroy(h);
      return DYCORE_EUNSUPPORTED;
    }
    ok = hipMalloc((void**)&h->ftiles, sizeof(AatItem) * ft.size()) == hipSuccess;
    ok = ok && hipMemcpy(h->ftiles, ft.data(), sizeof(AatItem) * ft.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (ok) {
      h->nftiles = (int)ft.size();
      h->ftblock = fblk;
      h->bytes += sizeof(AatItem) * ft.size() + sizeof(double) * 4 * nz;
    }
    std::vector<AatItem> at, pt;
    const int pblock = h->block;
    advect_tiles_split(nx, ny, h->M, h->Mv, h->block, at, pt);
    h->awide = 0;
    const size_t nall = at.size() + pt.size();
    ok = ok && hipMalloc((void**)&h->atiles, sizeof(AatItem) * nall) == hipSuccess;
    ok = ok && hipMemcpy(h->atiles, at.data(), sizeof(AatItem) * at.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (ok && !pt.empty())
      ok = hipMemcpy(h->atiles + at.size(), pt.data(), sizeof(AatItem) * pt.size(), hipMemcpyHostToDevice) ==
           hipSuccess;
    if (ok) {
      h->natiles = (int)at.size();
      h->nptiles = (int)pt.size();
      h->pblock = pblock;
      h->bytes += sizeof(AatItem) * nall;
    }
  }
  if (ok && !(h->flags & DYCORE_FORWARD_ONLY)) {
    h->adj_bytes = dyc_adjoint_workspace_bytes(h);
    ok = hipMalloc(&h->adj, h->adj_bytes) == hipSuccess;
    std::vector<AatItem> items;
    int blk = 0;
    if (ok && aat_items(nx, ny, h->M, items, blk)) {
      // rows 2..ny-2, then rows 1 and ny-1 (at the same block), which read the pole rows' sums and
      // so launch after them: the pole rows' chain then runs beside the others' launch
      std::vector<AatItem> mi, ei;
      const std::vector<int> hl = adapt_halos(h->M);
      int nmain = (int)items.size(), nedge = 0;
      const bool overlap = !(h->flags & DYCORE_SINGLE_STREAM) && (size_t)nx * ny * nz >= kAdjOverlapPoints;
      if (overlap && zonal_tiles(nx, row_range(2, ny - 2), hl, blk, mi) &&
          zonal_tiles(nx, {1, ny - 1}, hl, blk, ei)) {
        nmain = (int)mi.size();
        nedge = (int)ei.size();
        items = mi;
        items.insert(items.end(), ei.begin(), ei.end());
      }
      ok = hipMalloc((void**)&h->aat, sizeof(AatItem) * items.size()) == hipSuccess;
      ok = ok && hipMemcpy(h->aat, items.data(), sizeof(AatItem) * items.size(), hipMemcpyHostToDevice) ==
                     hipSuccess;
      if (ok) {
        h->aat_n = nmain;
        h->aat_edge_n = nedge;
        h->aat_block = blk;
        h->adj_bytes += sizeof(AatItem) * items.size();
      }
    }
    std::vector<AatItem> at;
    int ab = 0, pn = 0, psn = 0;
    if (ok && adt_items(nx, ny, h->M, h->Mv, at, ab, pn, psn)) {
      ok = hipMalloc((void**)&h->adt, sizeof(AatItem) * at.size()) == hipSuccess;
      ok = ok && hipMemcpy(h->adt, at.data(), sizeof(AatItem) * at.size(), hipMemcpyHostToDevice) == hipSuccess;
      if (ok) {
        h->adt_n = (int)at.size();
        h->adt_block = ab;
        h->adt_pp_n = pn;
        h->adt_pp_s = psn;
        h->adj_bytes += sizeof(AatItem) * at.size();
      }
    }
  }
  // a second stream (default priority): the forward advection's band tiles run there beside its
  // polar tiles, the adaptation adjoint's pole-row chain beside its row-fused launch.  The fork and
  // join events order work of one device: they need no system-scope fence (the host never waits on
  // them), which would write back and invalidate the caches at every fork and join.
  if (ok && !(h->flags & DYCORE_SINGLE_STREAM) &&
      (h->nptiles > 0 || (!(h->flags & DYCORE_FORWARD_ONLY) && (size_t)nx * ny * nz >= kAdjOverlapPoints))) {
    const unsigned ef = hipEventDisableTiming | hipEventDisableSystemFence;
    ok = hipStreamCreateWithFlags(&h->side.s, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&h->side.fork, ef) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&h->side.join, ef) == hipSuccess;
  }
  if (ok && (h->flags & DYCORE_LOWLAT_FILTERS)) {
    const std::vector<FiltItem> fi = filter_items(ny);
    if (!fi.empty()) {
      ok = hipMalloc((void**)&h->filt, sizeof(FiltItem) * fi.size()) == hipSuccess;
      ok = ok && hipMemcpy(h->filt, fi.data(), sizeof(FiltItem) * fi.size(), hipMemcpyHostToDevice) == hipSuccess;
      if (ok) h->nfilt = (int)fi.size();
    }
  }
  if (!ok) { dycore_destroy(h); return DYCORE_ENOMEM; }
  h->bytes += 2 * h->state_bytes + sizeof(double) * (kPoleSlots * 2 * (nz + 1) + 3 * (ny + 1) + 2) + 8 + h->adj_bytes;
  *out = h;
  return DYCORE_OK;
}

int dycore_kernel_timer_start(dycore_t h, int max_launches) {
  if (!h || max_launches < 1 || max_launches > 65536) return DYCORE_EINVAL;
  release_timer(h);
  dyc::KTimer& t = h->timer;
  t.ev = new (std::nothrow) hipEvent_t[2 * (size_t)max_launches];
  if (!t.ev) return DYCORE_ENOMEM;
  for (int q = 0; q < 2 * max_launches; ++q) {
    if (hipEventCreate(&t.ev[q]) != hipSuccess) {
      t.cap = q / 2;   // whole pairs made so far; the odd one out is destroyed here
      if (q % 2) (void)hipEventDestroy(t.ev[q - 1]);
      release_timer(h);
      return DYCORE_EHIP;
    }
  }
  t.cap = max_launches;
  t.n = 0;
  t.armed = 1;
  return DYCORE_OK;
}

int dycore_kernel_timer_stop(dycore_t h, double* total_ms, int* launches) {
  if (!h || !total_ms || !launches) return DYCORE_EINVAL;
  dyc::KTimer& t = h->timer;
  if (!t.ev) return DYCORE_EINVAL;
  t.armed = 0;
  double sum = 0;
  int st = DYCORE_OK;
  for (int q = 0; q < t.n; ++q) {
    float ms = 0;
    if (hipEventSynchronize(t.ev[2 * q + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, t.ev[2 * q], t.ev[2 * q + 1]) != hipSuccess) {
      st = DYCORE_EHIP;
      break;
    }
    sum += ms;
  }
  *total_ms = sum;
  *launches = st == DYCORE_OK ? t.n : 0;
  release_timer(h);
  return st;
}

int dycore_destroy(dycore_t h) {
  if (!h) return DYCORE_EINVAL;
  (void)hipDeviceSynchronize();
  if (h->geo) (void)hipFree(h->geo);
  if (h->scratch) (void)hipFree(h->scratch);
  if (h->pole) (void)hipFree(h->pole);
  if (h->diag) (void)hipFree(h->diag);
  if (h->count) (void)hipFree(h->count);
  if (h->adj) (void)hipFree(h->adj);
  if (h->aat) (void)hipFree(h->aat);
  if (h->adt) (void)hipFree(h->adt);
  if (h->filt) (void)hipFree(h->filt);
  if (h->ftiles) (void)hipFree(h->ftiles);
  if (h->atiles) (void)hipFree(h->atiles);
  if (h->side.fork) (void)hipEventDestroy(h->side.fork);
  if (h->side.join) (void)hipEventDestroy(h->side.join);
  if (h->side.s) (void)hipStreamDestroy(h->side.s);
  if (h->cap) (void)hipFree(h->cap);
  release_timer(h);
  delete h;
  return DYCORE_OK;
}

int dycore_step(dycore_t h, void* U, void* V, void* Phi, void* ps, int nsteps, void* stream) {
  if (!h || !U || !V || !Phi || !ps || nsteps < 0) return DYCORE_EINVAL;
  if (!aligned16(U) || !aligned16(V) || !aligned16(Phi) || !aligned16(ps)) return DYCORE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->prec == DYCORE_FP32)
    return step_impl<float>(h, (float*)U, (float*)V, (float*)Phi, (float*)ps, nsteps, s);
  return step_impl<double>(h, (double*)U, (double*)V, (double*)Phi, (double*)ps, nsteps, s);
}

int dycore_process_run(dycore_t h, int process, int n_rk, double hstep, void* U, void* V, void* Phi, void* ps,
                       void* stream) {
  if (!h || (process != 0 && process != 1) || n_rk < 0 || !(hstep > 0.0)) return DYCORE_EINVAL;
  if (!U || !V || !Phi || !ps || !aligned16(U) || !aligned16(V) || !aligned16(Phi) || !aligned16(ps))
    return DYCORE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->prec == DYCORE_FP32)
    return process_run_impl<float>(h, process, n_rk, hstep, (float*)U, (float*)V, (float*)Phi, (float*)ps, s);
  return process_run_impl<double>(h, process, n_rk, hstep, (double*)U, (double*)V, (double*)Phi, (double*)ps, s);
}

int dycore_stage(dycore_t h, int process, double ch, const void* bU, const void* bV, const void* bPhi,
                 const void* bps, const void* U, const void* V, const void* Phi, const void* ps, void* oU, void* oV,
                 void* oPhi, void* ops, void* stream) {
  if (!h || (process != 0 && process != 1)) return DYCORE_EINVAL;
  const void* ptrs[12] = {bU, bV, bPhi, bps, U, V, Phi, ps, oU, oV, oPhi, ops};
  for (auto p : ptrs)
    if (!p || !aligned16(p)) return DYCORE_EINVAL;
  if (oU == U || oV == V || oPhi == Phi || ops == ps) return DYCORE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->prec == DYCORE_FP32)
    return stage_impl<float>(h, process, ch, (const float*)bU, (const float*)bV, (const float*)bPhi,
                             (const float*)bps, (const float*)U, (const float*)V, (const float*)Phi,
                             (const float*)ps, (float*)oU, (float*)oV, (float*)oPhi, (float*)ops, s);
  return stage_impl<double>(h, process, ch, (const double*)bU, (const double*)bV, (const double*)bPhi,
                            (const double*)bps, (const double*)U, (const double*)V, (const double*)Phi,
                            (const double*)ps, (double*)oU, (double*)oV, (double*)oPhi, (double*)ops, s);
}

int dycore_diagnostics(dycore_t h, const void* U, const void* V, const void* Phi, const void* ps, double* mass_out,
                       double* energy_out, void* stream) {
  if (!h || !U || !V || !Phi || !ps || !mass_out || !energy_out) return DYCORE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* sums = h->diag + 3 * (h->ny + 1);
  hipError_t e;
  if (h->prec == DYCORE_FP32)
    e = launch_diag<float>(h->g, (const float*)U, (const float*)V, (const float*)Phi, (const float*)ps, h->diag,
                           sums, s);
  else
    e = launch_diag<double>(h->g, (const double*)U, (const double*)V, (const double*)Phi, (const double*)ps,
                            h->diag, sums, s);
  if (e != hipSuccess) return DYCORE_EHIP;
  double out[2];
  if (hipMemcpyAsync(out, sums, sizeof(out), hipMemcpyDeviceToHost, s) != hipSuccess) return DYCORE_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return DYCORE_EHIP;
  *mass_out = out[0];
  *energy_out = out[1];
  return DYCORE_OK;
}

int dycore_diagnostics_noalloc(dycore_t h, const void* U, const void* V, const void* Phi, const void* ps,
                               double* out_dev, void* stream) {
  if (!h || !U || !V || !Phi || !ps || !out_dev) return DYCORE_EINVAL;
  if (h->ny + 1 > kNoallocMaxRows) return DYCORE_EINVAL;
  double* part = (h->device >= 0 && h->device < kMaxDevices) ? g_scratch_dev[h->device] : nullptr;
  if (!part) return DYCORE_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (h->prec == DYCORE_FP32)
    e = launch_diag<float>(h->g, (const float*)U, (const float*)V, (const float*)Phi, (const float*)ps, part,
                           out_dev, s);
  else
    e = launch_diag<double>(h->g, (const double*)U, (const double*)V, (const double*)Phi, (const double*)ps,
                            part, out_dev, s);
  return hip_status(e);
}

int dycore_check_finite(dycore_t h, const void* U, const void* V, const void* Phi, const void* ps,
                        long long* count_out, void* stream) {
  if (!h || !U || !V || !Phi || !ps) return DYCORE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_zero<unsigned long long>(h->count, 1, s);
  const void* f[4] = {U, V, Phi, ps};
  const size_t n[4] = {h->nU, h->nV, h->nF, h->nP};
  for (int q = 0; q < 4 && e == hipSuccess; ++q)
    e = (h->prec == DYCORE_FP32) ? launch_nonfinite<float>((const float*)f[q], n[q], h->count, s)
                                 : launch_nonfinite<double>((const double*)f[q], n[q], h->count, s);
  if (e != hipSuccess) return DYCORE_EHIP;
  unsigned long long c = 0;
  if (hipMemcpyAsync(&c, h->count, sizeof(c), hipMemcpyDeviceToHost, s) != hipSuccess) return DYCORE_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return DYCORE_EHIP;
  if (count_out) *count_out = (long long)c;
  return c ? DYCORE_ENONFINITE : DYCORE_OK;
}

int dycore_leap_table(dycore_t h, int* m_rows, int* m_vrows) {
  if (!h) return DYCORE_EINVAL;
  if (m_rows) std::memcpy(m_rows, h->M.data(), sizeof(int) * h->M.size());
  if (m_vrows) std::memcpy(m_vrows, h->Mv.data(), sizeof(int) * h->Mv.size());
  return DYCORE_OK;
}

int dycore_substeps(dycore_t h) { return h ? h->msub : DYCORE_EINVAL; }
int dycore_block(dycore_t h) { return h ? h->block : DYCORE_EINVAL; }
size_t dycore_workspace_bytes(dycore_t h) { return h ? h->bytes : 0; }

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// Batches: members of mixed grids advance together, one persistent launch per global stage.
// ------------------------------------------------------------------------------------------------
namespace {

struct PrepDesc {
  int nx, ny, nz, pad;
  const void* F;
  const void* P;
  double* pole;
};

template <typename T>
__global__ void k_prep_batch(const PrepDesc* d, int n) {
  // block (m, v): member m, value v of its 2*(nz+1) pole values; one wavefront each
  const int m = blockIdx.y;
  if (m >= n) return;
  const PrepDesc pd = d[m];
  const int v = blockIdx.x;
  if (v >= 2 * (pd.nz + 1)) return;
  const int p = v / (pd.nz + 1), k = v % (pd.nz + 1);
  const int j = (p == 0) ? 0 : pd.ny;
  const T* src = (k < pd.nz) ? (const T*)pd.F + ((size_t)j * pd.nz + k) * pd.nx : (const T*)pd.P + (size_t)j * pd.nx;
  double s = 0;
  for (int i = threadIdx.x; i < pd.nx; i += 64) s += (double)src[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x == 0) pd.pole[p * (pd.nz + 1) + k] = s / (double)pd.nx;
}

template <typename T>
int batch_build(dycore_batch_s* b) {
  const int n = b->n;
  // every member's adaptation tiles for the batch's block, one table after the other
  std::vector<AatItem> tiles;
  std::vector<size_t> toff(n), aoff(n);
  std::vector<int> tcount(n), acount(n);
  for (int m = 0; m < n; ++m) {
    const dycore_s* h = b->hs[m];
    std::vector<AatItem> t, at;
    if (!aat_tiles(h->nx, h->ny, h->M, b->block, t, 0, h->ny)) return DYCORE_EUNSUPPORTED;
    advect_tiles(h->nx, h->ny, h->M, h->Mv, b->block, at);
    toff[m] = tiles.size();
    tcount[m] = (int)t.size();
    tiles.insert(tiles.end(), t.begin(), t.end());
    aoff[m] = tiles.size();
    acount[m] = (int)at.size();
    tiles.insert(tiles.end(), at.begin(), at.end());
  }
  if (hipMalloc((void**)&b->d_tiles, sizeof(AatItem) * tiles.size()) != hipSuccess) return DYCORE_ENOMEM;
  if (hipMemcpy(b->d_tiles, tiles.data(), sizeof(AatItem) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess)
    return DYCORE_EHIP;
  std::vector<StageArgs<T>> args((size_t)b->nstage_max * n);
  for (int m = 0; m < n; ++m) {
    dycore_s* h = b->hs[m];
    T* U = (T*)b->U[m]; T* V = (T*)b->V[m]; T* F = (T*)b->F[m]; T* P = (T*)b->P[m];
    const int nst = 3 * (h->msub + 1);
    for (int sidx = 0; sidx < b->nstage_max; ++sidx) {
      StageArgs<T>& a = args[(size_t)sidx * n + m];
      if (sidx < nst) {
        a = step_stage_args<T>(h, sidx / 3, sidx % 3, U, V, F, P);
      } else {
        a = make_args<T>(h, -1, 0.0, U, V, F, P, U, V, F, P, U, V, F, P, nullptr, nullptr, nullptr);
      }
      a.tiles = b->d_tiles + toff[m];
      a.ntiles = tcount[m];
      a.tblock = b->block;
      a.atiles = b->d_tiles + aoff[m];
      a.natiles = acount[m];
      a.ablock = b->block;
      a.awide = 1;
      a.ptiles = nullptr;
      a.nptiles = 0;
    }
  }
  if (hipMalloc(&b->d_args, sizeof(StageArgs<T>) * args.size()) != hipSuccess) return DYCORE_ENOMEM;
  if (hipMemcpy(b->d_args, args.data(), sizeof(StageArgs<T>) * args.size(), hipMemcpyHostToDevice) != hipSuccess)
    return DYCORE_EHIP;
  // work items: members largest first, rows in XCD order, each member padded to a multiple of 8
  std::vector<int> order(n);
  for (int m = 0; m < n; ++m) order[m] = m;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const dycore_s* a = b->hs[x]; const dycore_s* c = b->hs[y];
    return (size_t)a->nx * a->nz > (size_t)c->nx * c->nz;
  });
  // tiles in member order; each table is a multiple of 8 long and XCD-ordered, so item w still runs
  // on XCD w mod 8 in the persistent launch (whose grid is a multiple of 8)
  std::vector<int2> items, titems;
  for (int m : order)
    for (int q = 0; q < acount[m]; ++q) items.push_back(int2{m, q});
  b->nitems = (int)items.size();
  for (int m : order)
    for (int q = 0; q < tcount[m]; ++q) titems.push_back(int2{m, q});
  b->ntitems = (int)titems.size();
  if (hipMalloc((void**)&b->d_titems, sizeof(int2) * titems.size()) != hipSuccess) return DYCORE_ENOMEM;
  if (hipMemcpy(b->d_titems, titems.data(), sizeof(int2) * titems.size(), hipMemcpyHostToDevice) != hipSuccess)
    return DYCORE_EHIP;
  if (hipMalloc((void**)&b->d_items, sizeof(int2) * items.size()) != hipSuccess) return DYCORE_ENOMEM;
  if (hipMemcpy(b->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice) != hipSuccess)
    return DYCORE_EHIP;
  std::vector<PrepDesc> pd(n);
  for (int m = 0; m < n; ++m) {
    dycore_s* h = b->hs[m];
    pd[m] = PrepDesc{h->nx, h->ny, h->nz, 0, b->F[m], b->P[m], pole_slot(h, 0)};
  }
  if (hipMalloc(&b->d_prep, sizeof(PrepDesc) * n) != hipSuccess) return DYCORE_ENOMEM;
  if (hipMemcpy(b->d_prep, pd.data(), sizeof(PrepDesc) * n, hipMemcpyHostToDevice) != hipSuccess) return DYCORE_EHIP;
  return DYCORE_OK;
}

template <typename T>
int batch_step(dycore_batch_s* b, int nsteps, hipStream_t s) {
  int maxnz = 0;
  for (auto h : b->hs) maxnz = std::max(maxnz, h->nz);
  hipLaunchKernelGGL((k_prep_batch<T>), dim3(2 * (maxnz + 1), b->n), dim3(64), 0, s, (const PrepDesc*)b->d_prep,
                     b->n);
  if (hipGetLastError() != hipSuccess) return DYCORE_EHIP;
  const StageArgs<T>* args = static_cast<const StageArgs<T>*>(b->d_args);
  for (int n = 0; n < nsteps; ++n) {
    for (int sidx = 0; sidx < b->nstage_max; ++sidx) {
      hipError_t e = launch_stage_batch<T>(args + (size_t)sidx * b->n, b->n, b->max_nz, b->d_titems, b->ntitems,
                                           b->d_items, b->nitems, b->grid, b->block, b->lds, s);
      if (e != hipSuccess) return DYCORE_EHIP;
    }
    for (int m = 0; m < b->n; ++m) {   // members with the low-latitude filters close their step
      const dycore_s* h = b->hs[m];
      if (launch_lowlat<T>(h->g, h->filt, h->nfilt, (T*)b->U[m], (T*)b->V[m], (T*)b->F[m], (T*)b->P[m], s) !=
          hipSuccess)
        return DYCORE_EHIP;
    }
  }
  return DYCORE_OK;
}

}  // namespace

extern "C" {

int dycore_batch_create(int n, const dycore_t* hs, void* const* U, void* const* V, void* const* Phi,
                        void* const* ps, int block, int grid, dycore_batch_t* out) {
  if (!out || n < 1 || !hs || !U || !V || !Phi || !ps) return DYCORE_EINVAL;
  *out = nullptr;
  const int prec = hs[0] ? hs[0]->prec : -1;
  int max_nx = 0, nst = 0;
  for (int m = 0; m < n; ++m) {
    if (!hs[m] || hs[m]->prec != prec || !U[m] || !V[m] || !Phi[m] || !ps[m]) return DYCORE_EINVAL;
    if (!aligned16(U[m]) || !aligned16(V[m]) || !aligned16(Phi[m]) || !aligned16(ps[m])) return DYCORE_EINVAL;
    for (int q = 0; q < m; ++q)
      if (hs[q] == hs[m]) return DYCORE_EINVAL;   // each member needs its own scratch
    max_nx = std::max(max_nx, hs[m]->nx);
    nst = std::max(nst, 3 * (hs[m]->msub + 1));
  }
  if (block == 0) block = 256;
  if (block < 64 || block > 1024 || block % 64) return DYCORE_EINVAL;
  if (block > kBatchMaxBlock) return DYCORE_EUNSUPPORTED;
  const int el = prec == DYCORE_FP32 ? 4 : 8;
  const size_t lds = std::max(adapt_tile_lds_bytes(block, el), advect_tile_lds_bytes(block, el));
  int max_nz = 0;
  for (int m = 0; m < n; ++m) max_nz = std::max(max_nz, hs[m]->nz);
  if (lds > 160 * 1024) return DYCORE_EUNSUPPORTED;
  dycore_batch_s* b = new (std::nothrow) dycore_batch_s();
  if (!b) return DYCORE_ENOMEM;
  b->n = n; b->prec = prec; b->block = block; b->max_nx = max_nx; b->nstage_max = nst; b->lds = lds;
  b->max_nz = max_nz;
  b->hs.assign(hs, hs + n);
  b->U.assign(U, U + n); b->V.assign(V, V + n); b->F.assign(Phi, Phi + n); b->P.assign(ps, ps + n);
  const int st = prec == DYCORE_FP32 ? batch_build<float>(b) : batch_build<double>(b);
  if (st != DYCORE_OK) { dycore_batch_destroy(b); return st; }
  if (grid <= 0) {
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int per_cu = (int)std::max<size_t>(1, (160 * 1024) / lds);
    per_cu = std::min(per_cu, std::max(1, 2048 / block));
    grid = cus * per_cu;
  }
  grid = std::max(8, grid / 8 * 8);
  b->grid = std::min(grid, (b->nitems + 7) / 8 * 8);
  *out = b;
  return DYCORE_OK;
}

int dycore_batch_step(dycore_batch_t b, int nsteps, void* stream) {
  if (!b || nsteps < 0) return DYCORE_EINVAL;
  if (nsteps == 0) return DYCORE_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return b->prec == DYCORE_FP32 ? batch_step<float>(b, nsteps, s) : batch_step<double>(b, nsteps, s);
}

int dycore_batch_destroy(dycore_batch_t b) {
  if (!b) return DYCORE_EINVAL;
  (void)hipDeviceSynchronize();
  if (b->d_args) (void)hipFree(b->d_args);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_titems) (void)hipFree(b->d_titems);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->d_prep) (void)hipFree(b->d_prep);
  delete b;
  return DYCORE_OK;
}

}  // extern "C"
