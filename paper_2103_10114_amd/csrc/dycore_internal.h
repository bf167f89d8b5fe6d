// Internal declarations shared by the HIP translation units of libdycore.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

struct dycore_s;

namespace dyc {

// Geometry and constants as the kernels see them (device pointers to FP64 tables).
struct GeoDev {
  int nx, ny, nz;
  double a, omega, g, rd, cp, p0, t0, kappa, b, dlam, dth, acap, RT0;
  double kstar;         // p_s diffusion coefficient kappa* (m^2/s), 0 = off
  const double* s;      // sin(theta_j), rows 0..ny
  const double* cot;    // cot(theta_j)
  const double* f;      // 2 Omega cos(theta_j)
  const int* M;         // leap span per scalar/U row (odd, 1 at the poles)
  const double* sv;     // sin(theta_{j+1/2}), V rows 0..ny-1
  const double* cotv;
  const double* fv;
  const int* Mv;        // leap span per V row
  const double* sigh;   // nz+1 half levels
  const double* sig;    // nz full levels
  const double* dsig;   // nz layer thickness
  const double* cl;     // ln(sigh[l+1]/sigh[l]) for l >= 1, 0 for l = 0
  const double* cpk;    // ln(sigh[k+1]/sig[k])
  const double* phis;   // (ny+1)*nx surface geopotential, pole rows = row mean
};

// Difference factors as the forward stages multiply by them, rounded to the field precision
// (device tables; used by the adjoint kernels, kept out of GeoDev so that the forward kernels'
// arguments stay small).
struct GeoFac {
  const double* rdx;    // scalar/U rows: 1 / (M a sin(theta) dlam), 0 at the poles
  const double* rdy;    // scalar/U rows: 1 / (a sin(theta) dtheta), 0 at the poles
  const double* rdxv2;  // V rows: 1 / (2 Mv a sin(theta) dlam)
  const double* rdyv2;  // V rows: 1 / (2 a sin(theta) dtheta)
  const double* r2d;    // levels: 1 / (2 dsigma)
  const double* rsig;   // levels: 1 / sigma (correctly rounded, as a division on the device)
};

// Live timing of one kernel's launches: HIP events recorded on the launch stream right before
// and after each launch, up to `cap` launches.
struct KTimer {
  int armed = 0, n = 0, cap = 0;
  hipEvent_t* ev = nullptr;   // 2 cap events: start and end of each timed launch
};

// Pole slot layout: double[2][nz+1]; [p][k] = Phi pole value at level k, [p][nz] = p_s pole value,
// p = 0 north, 1 south.

// Zonal tiles of the tiled adaptation stage and its adjoint: one work item per (row, tile), a tile
// being w owned columns from i0 plus a halo of hl = n_j + 1 columns on each side (n_j the row's leap
// half width), one column per thread, w + 2 hl <= the launch's block.  Items are ordered so that the
// workgroups one XCD runs cover a contiguous band of rows; padding items have j = -1.
struct AatItem {
  int j, i0, w, hl;
};
constexpr int kMaxLevels = 128;         // most model levels a handle takes
// Grids of at least this many points run the stage adjoints' pole-row chains beside their row-fused
// launches (on smaller grids a fork and join cost more than the chain they would hide).
constexpr size_t kAdjOverlapPoints = size_t(1) << 24;
constexpr int kAatMaxBlock = 320;       // adjoint tiles
constexpr int kFwdTileMaxBlock = 1024;  // forward adaptation tiles
constexpr int kBatchMaxBlock = 512;     // the persistent batched stage (its VGPR budget: 256)

// One stage out = base + ch * T(in) of one member.
template <typename T>
struct StageArgs {
  GeoDev g;
  const T* inU; const T* inV; const T* inF; const T* inP;
  const T* bU; const T* bV; const T* bF; const T* bP;
  T* oU; T* oV; T* oF; T* oP;
  const double* pin;    // pole values of `in`
  const double* pbase;  // pole values of `base`
  double* pout;         // pole values written for `out`
  double ch;
  int process;          // 0 adaptation, 1 advection, -1 idle
  int pad;
  const AatItem* tiles;  // zonal tiles of the adaptation stage (rows 0..ny)
  double* cap;          // [2 poles][2][nz] FP64 cap sums of the stage's input (either process)
  int ntiles;           // tile count (a multiple of 8)
  int tblock;           // threads per tile workgroup
  const AatItem* atiles; // zonal tiles of the advection stage (rows 0..ny; hl < 0: wide form)
  int natiles;          // their count (a multiple of 8)
  int ablock;           // threads per advection tile workgroup
  int awide;            // 1 if atiles holds wide-form items
  const AatItem* ptiles; // single-member launches: wide tiles of the rows whose halos do not fit
  int nptiles;          // the workgroup (next to the poles), a second launch of pblock threads
  int pblock;
};

// A second stream for launches that overlap another of the same stage (the advection's band tiles
// run there beside its polar tiles; the adaptation adjoint's pole-row chain beside its row-fused
// launch): the stage's stream forks to it and joins it again through the two events (default
// priority).
struct SideLaunch {
  hipStream_t s;
  hipEvent_t fork, join;
};

// Adjoint of one stage about `in`.
template <typename T>
struct AdjArgs {
  GeoDev g;
  const T* inU; const T* inV; const T* inF; const T* inP;      // linearisation state
  const T* aoU; const T* aoV; const T* aoF; const T* aoP;      // adjoint of the stage output
  T* abU; T* abV; T* abF; T* abP;                             // += adjoint of base
  T* aiU; T* aiV; T* aiF; T* aiP;                             // += adjoint of in
  const double* pin;   // pole values of `in`
  double ch;
  int process;
  int pad;
  // workspace (device), sized at create
  T* w3[16];           // 3D scratch fields, (ny+1)*(nz+1)*nx entries each
  T* w2[8];            // 2D scratch fields, (ny+1)*nx entries each
  double* wpole;       // pole scratch, 64*(nz+1) doubles
};

// One zonal row the low-latitude filters act on: field 0 U, 1 V, 2 Phi, 3 p_s; row j; r < 0 for the
// simplified filter (removes the 2-dlam wave), r > 0 for the 3-point operator's coefficient.
struct FiltItem {
  int field, j;
  double r;
};

// Launch helpers implemented in the kernel translation units.
template <typename T>
hipError_t launch_pole_prep(const GeoDev& g, const T* F, const T* ps, double* pole, hipStream_t s);
// One stage out = base + ch T(in): the pole cap sums of `in`, then the process's zonal tiles.
template <typename T>
hipError_t launch_stage(const StageArgs<T>& a, hipStream_t s, const SideLaunch* side = nullptr);
// One batched stage: the cap sums of every member, then a persistent launch over the adaptation
// tiles (titems) and one over the advection tiles (items) of every member.
template <typename T>
hipError_t launch_stage_batch(const StageArgs<T>* d_args, int nargs, int max_nz, const int2* d_titems, int ntitems,
                              const int2* d_items, int nitems, int grid, int block, size_t lds, hipStream_t s);
template <typename T>
hipError_t launch_stage_adjoint(const AdjArgs<T>& a, int block, hipStream_t s);
// FP64 mass and energy: per-row partials (3 (ny+1) doubles in `partial`), then their fixed-order
// sum into out[0] (mass) and out[1] (energy), both device memory.
template <typename T>
hipError_t launch_diag(const GeoDev& g, const T* U, const T* V, const T* F, const T* ps,
                       double* partial, double* out, hipStream_t s);
template <typename T>
hipError_t launch_nonfinite(const T* x, size_t n, unsigned long long* count, hipStream_t s);
// The low-latitude filters on the rows of `items` (every level of the 3D fields), in place.
template <typename T>
hipError_t launch_lowlat(const GeoDev& g, const FiltItem* items, int nitems, T* U, T* V, T* F, T* P,
                         hipStream_t s);
template <typename T>
hipError_t launch_axpy_fill(T* dst, const T* src, size_t n, hipStream_t s);   // dst = src (copy) via kernel
template <typename T>
hipError_t launch_zero(T* dst, size_t n, hipStream_t s);

size_t adapt_tile_lds_bytes(int block, int elem);    // LDS of an adaptation tile workgroup
size_t advect_tile_lds_bytes(int block, int elem);   // LDS of an advection tile workgroup

// A uniform row of a global array: the array base (the kernel argument's, one SGPR pair for every
// row) plus a uniform 32-bit element offset made opaque with readfirstlane (one SGPR per row; loop
// strength reduction would otherwise keep one 64-bit address per array and owned column in VGPRs).
// Indexed by a 32-bit column, every access is a global load or store of base + 32-bit VGPR byte
// offset (a generic pointer would make it a flat access).  Arrays are limited to 2^32 bytes.
template <typename T>
struct ORow {
  __attribute__((address_space(1))) T* p;
  unsigned o;
  __device__ __forceinline__ __attribute__((address_space(1))) T& operator[](unsigned i) const {
    return *(__attribute__((address_space(1))) T*)(
        reinterpret_cast<__attribute__((address_space(1))) const char*>(p) + (o + i) * (unsigned)sizeof(T));
  }
};
template <typename T>
__device__ __forceinline__ ORow<T> urow(T* base, size_t off) {
  return ORow<T>{(__attribute__((address_space(1))) T*)base, (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)off)};
}

// XCD-aware row order: workgroups are dispatched round-robin over the 8 XCDs,
// so block b lands on XCD b % 8.  Give each XCD a contiguous band of rows, in
// order, so that neighbouring rows (which share halo rows) share an L2.
__device__ __forceinline__ int xcd_row(int b, int nrows) {
  const int x = b & 7, slot = b >> 3;
  const int q = nrows >> 3, rem = nrows & 7;
  const int start = x * q + (x < rem ? x : rem);
  return start + slot;
}

// XCD-aware order for a (column tile, level, row) grid launched as dim3(gx, nz, nrows): the
// linear block index goes round-robin over the XCDs; each XCD gets a contiguous band of the
// (row, level, tile) tuples, row slowest, so that the rows a point reads around it (j-1, j+1)
// are mostly in the same L2.
__device__ __forceinline__ void xcd_tile3(int gx, int nz, int nrows, int& x, int& k, int& j) {
  const int b = (int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z));
  const int total = gx * nz * nrows;
  const int xc = b & 7, slot = b >> 3;
  const int q = total >> 3, rem = total & 7;
  const int tup = xc * q + (xc < rem ? xc : rem) + slot;
  x = tup % gx;
  k = (tup / gx) % nz;
  j = tup / (gx * nz);
}



// As xcd_tile3, with the levels in blocks of KB (KB divides nz): the tuples run (level block, row,
// level in the block, tile), tile fastest, so that a point's neighbours at rows j+-1 and levels k+-1
// were read a few dozen workgroups earlier on the same XCD, and the working set of the rows in
// flight (every field a point reads, KB levels deep) stays well inside an XCD's L2.
__device__ __forceinline__ void xcd_tile3_kb(int gx, int nz, int nrows, int KB, int& x, int& k, int& j) {
  const int b = (int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z));
  const int total = gx * nz * nrows;
  const int xc = b & 7, slot = b >> 3;
  const int q = total >> 3, rem = total & 7;
  const int tup = xc * q + (xc < rem ? xc : rem) + slot;
  const int per_block = nrows * KB * gx;
  const int kb = tup / per_block, r = tup - kb * per_block;
  j = r / (KB * gx);
  const int r2 = r - j * (KB * gx);
  k = kb * KB + r2 / gx;
  x = r2 % gx;
}

// What the adjoint translation unit sees of a handle.
struct HandleView {
  GeoDev g;
  int prec, msub;
  double dt;
  size_t nU, nV, nF, nP, elem, state_bytes;
  void* adj;
  size_t adj_bytes;
  double* pole;      // pole slots of the handle
  void* scratch;     // forward scratch y1, y2
  int block;
  GeoFac fac;
  int* recorded;     // 1 while the adjoint workspace holds the stage inputs of a recorded step
  KTimer* timer;     // launches of the row-fused adaptation-stage adjoint kernel
  const AatItem* aat;   // tiled adaptation-adjoint work items (device), or NULL when rows do not fit
  int aat_n;            // item count (a multiple of 8)
  int aat_block;        // threads per tile workgroup
  int aat_edge_n;       // > 0: aat holds rows 2..ny-2, then this many items of rows 1 and ny-1
  const AatItem* adt;   // tiled advection-adjoint work items (device), or NULL: per-point kernels
  int adt_n, adt_block; // their count (a multiple of 8) and workgroup size (up to 256)
  int adt_pp_n, adt_pp_s; // rows 1..pp_n and ny-pp_s..ny-1 go with the pole rows (per point)
  const FiltItem* filt; // rows of the low-latitude filters (device), NULL when they are off
  int nfilt;
  const AatItem* ftiles; // zonal tiles of the forward adaptation stage (device)
  int nftiles, ftblock;
  const AatItem* atiles; // zonal tiles of the forward advection stage (device)
  int natiles, ablock, awide;
  const AatItem* ptiles; // its polar tiles (larger workgroups), NULL when none
  int nptiles, pblock;
  const SideLaunch* side; // second stream: the forward advection's band tiles beside its polar tiles
  const SideLaunch* adj_side; // the same stream for the stage adjoints' pole-row chains (NULL: serial)
  double* cap;           // cap sums of the forward adaptation stage (device, 4 nz doubles)
};
HandleView view_of(const dycore_s* h);

}  // namespace dyc
