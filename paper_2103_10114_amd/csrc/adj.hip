// Adjoint (transpose) of one stage and of the outer step (gfx950).
//
// The adjoint is the transpose of the forward map under the Euclidean inner
// product over every stored entry.  Each stage adjoint first recomputes the
// column diagnostics of its input (P, l, q, the leaped d+l and d+q, R T',
// phi', divergence D, prefix sums S, sigma-dot, omega/p) into scratch, then
// runs the transposed operators in reverse order as gather kernels: every
// adjoint entry collects the contributions of all forward outputs that read it
// (the transpose of a leaped d+ is a leaped d- with mirrored offsets, of an
// average the mirrored average, of a prefix sum a suffix sum, of a pole read
// a spread of the row sum over the row).  No atomics: results are
// deterministic.  Column sums and pole sums are FP64.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/dycore.h"
#include "dycore_internal.h"

using namespace dyc;

namespace {

using C = double;

__device__ __forceinline__ int wrp(int i, int nx) { return i >= nx ? i - nx : (i < 0 ? i + nx : i); }
// one-sided forms, where the offset's sign is known: 0 <= i < 2 nx, and -nx <= i < nx
__device__ __forceinline__ int wrp_up(int i, int nx) { return i >= nx ? i - nx : i; }
__device__ __forceinline__ int wrp_dn(int i, int nx) { return i < 0 ? i + nx : i; }

__device__ __forceinline__ double wave_sum(double acc) {
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  return acc;
}

// One lane's FP64 partial sum of a row of n values: the lane's elements (lane, lane + 64, ...) added
// in index order, the loads of eight of them issued before their additions.
template <typename T>
__device__ __forceinline__ double lane_row_sum(const T* p, int n, int lane) {
  constexpr int CH = 8;
  double s = 0;
  for (int i0 = lane; i0 < n; i0 += 64 * CH) {
    T v[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) v[u] = p[i0 + 64 * u < n ? i0 + 64 * u : i0];
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (i0 + 64 * u < n) s += (double)v[u];
  }
  return s;
}

template <typename T> __device__ __forceinline__ T tsqrt(T x);
template <> __device__ __forceinline__ float tsqrt<float>(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double tsqrt<double>(double x) { return sqrt(x); }
template <typename T> __device__ __forceinline__ T tlog(T x);
template <> __device__ __forceinline__ float tlog<float>(float x) { return logf(x); }
template <> __device__ __forceinline__ double tlog<double>(double x) { return log(x); }

// Scratch of one stage adjoint.
template <typename T>
struct Scr {
  // forward recompute
  T *P, *L, *Q, *DL, *DQ;          // 2D (ny+1)*nx
  T *RT, *PHI, *D, *WP;            // 3D scalar
  T *S, *SD;                       // half levels (ny+1)*(nz+1)*nx
  // adjoint intermediates (3D, index like the scalar/U/V fields)
  T *AVGL, *AD, *AFE, *AP3, *HH, *FU, *AUU, *AUD, *MV, *FV, *UV, *AVV, *AVD, *APU3, *APV3;
  T *APHI, *ART, *AL3, *AQ3, *ADL3, *ADQ3;   // adaptation: per-point inputs of the column sums
  T *UA, *VT;                      // advection: u at U points, v sin(theta) at V points
  T *ASD;                          // half levels
  double *AP2, *APU2, *APV2, *AL2, *AQ2, *ADL2, *ADQ2, *APSR;   // 2D FP64
  double* psum;                    // pole sums [8][2][nz+1]
};

// Pole sums slots
enum { PS_AD = 0, PS_AVGL = 1, PS_AOF = 2, PS_AFE = 3 };

template <typename T>
struct Ctx {
  GeoDev g;
  const T *U, *V, *F, *P;          // linearisation state (stage input)
  const T *aoU, *aoV, *aoF, *aoP;  // adjoint of the stage output
  T *abU, *abV, *abF, *abP;        // += adjoint of base
  T *aiU, *aiV, *aiF, *aiP;        // += adjoint of in
  const double* pin;               // pole values of the linearisation state
  double ch;
  Scr<T> s;
  GeoFac f;                        // difference factors of the forward stages
  int jr0 = 0, jrs = 1;            // rows a launch covers: jr0 + jrs * (grid row index), or with
  int rsplit = 0;                  // rsplit > 0: grid rows r < rsplit are rows r, the rest the last
                                   // rows (ny - (grid rows - 1 - r))
  int blk = 0;                     // workgroup size of the row-fused kernel (the handle's)
  int parts = 7;                   // first adaptation transposes: 1 scalar point (+ suffix), 2 U, 4 V
  KTimer* timer = nullptr;         // host side: times the row-fused kernel's launches when armed
  const AatItem* aat = nullptr;    // work items of the tiled row-fused adaptation adjoint (NULL: per point)
  int aat_n = 0;                   // item count
  int aat_blk = 0;                 // threads per tile workgroup
  int aat_edge_n = 0;              // > 0: aat holds rows 2..ny-2, then this many items of rows 1 and
                                   // ny-1 (which read the pole rows' sums) for a launch of their own
  const SideLaunch* side = nullptr;   // second stream: the pole rows' chain runs there beside k_aat
  int f2d_ready = 0;               // s.P, L, Q, DL, DQ already hold this stage's 2D recompute
  const T* next_ps = nullptr;      // non-NULL: the chain ends with the next stage's 2D recompute (p_s
  const double* next_pin = nullptr;   // and pole values of its input) into the other set, next2d
  T* next2d[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const AatItem* adt = nullptr;    // work items of the tiled row-fused advection adjoint (NULL: per point)
  int adt_n = 0, adt_blk = 0;      // their count and workgroup size (rows with halos up to 112 columns)
  int pp_n = 0, pp_s = 0;          // with it: rows 1..pp_n and ny-pp_s..ny-1 (halos too wide for its
                                   // tiles) run the per-point kernels with the pole rows
  int fwd_all = 1;                 // forward recompute of R T', phi', omega/p too (0: D, S, sigma-dot only)
  int ai_zero = 0;                 // the input adjoint starts at zero and, in its interior rows, only the
                                   // row-fused kernel adds to it: those rows are stored without a read
                                   // (and need not be cleared by the caller)
  int base_in_tail = 0;            // advection with one base and input adjoint: the interior base transpose
                                   // is added by the column tail (k_l3, k_t3) instead of k_base
};

// The row of grid row r of a launch over nrows rows (Ctx::jr0, jrs, rsplit).
template <typename T>
__device__ __forceinline__ int row_of(const Ctx<T>& c, int r, int nrows) {
  if (c.rsplit > 0) return r < c.rsplit ? r : c.g.ny - (nrows - 1 - r);
  return c.jr0 + c.jrs * r;
}

template <typename T>
__device__ __forceinline__ size_t i3(const GeoDev& g, int j, int k, int i) {
  return ((size_t)j * g.nz + k) * g.nx + i;
}
template <typename T>
__device__ __forceinline__ size_t ih(const GeoDev& g, int j, int h, int i) {
  return ((size_t)j * (g.nz + 1) + h) * g.nx + i;
}

// 32-bit forms: a field holds fewer than 2^30 elements (create refuses larger grids), so element
// indices and byte offsets fit 32 bits and a load is the array's base plus a 32-bit offset
__device__ __forceinline__ unsigned i3u(const GeoDev& g, int j, int k, int i) {
  return (unsigned)((j * g.nz + k) * g.nx + i);
}
__device__ __forceinline__ unsigned ihu(const GeoDev& g, int j, int h, int i) {
  return (unsigned)((j * (g.nz + 1) + h) * g.nx + i);
}
template <typename T>
__device__ __forceinline__ T ldg(const T* p, unsigned idx) {
  return *(const __attribute__((address_space(1))) T*)(
      (const __attribute__((address_space(1))) char*)p + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stg(T* p, unsigned idx, T v) {
  *(__attribute__((address_space(1))) T*)((__attribute__((address_space(1))) char*)p + idx * (unsigned)sizeof(T)) = v;
}

// pole-aware reads of the linearisation state
template <typename T>
__device__ __forceinline__ T Fe(const Ctx<T>& c, int j, int k, int i) {
  const GeoDev& g = c.g;
  if (j == 0) return (T)c.pin[k];
  if (j == g.ny) return (T)c.pin[(g.nz + 1) + k];
  return ldg(c.F, i3u(g, j, k, i));
}
template <typename T>
__device__ __forceinline__ T Ue(const Ctx<T>& c, int j, int k, int i) {
  const GeoDev& g = c.g;
  if (j <= 0 || j >= g.ny) return T(0);
  return ldg(c.U, i3u(g, j, k, i));
}
template <typename T>
__device__ __forceinline__ T Ve(const Ctx<T>& c, int jv, int k, int i) {
  return ldg(c.V, i3u(c.g, jv, k, i));
}
template <typename T>
__device__ __forceinline__ T psE(const Ctx<T>& c, int j, int i) {
  const GeoDev& g = c.g;
  if (j == 0) return (T)c.pin[g.nz];
  if (j == g.ny) return (T)c.pin[(g.nz + 1) + g.nz];
  return c.P[(size_t)j * g.nx + i];
}
template <typename T>
__device__ __forceinline__ T P2(const Ctx<T>& c, int j, int i) { return c.s.P[(size_t)j * c.g.nx + i]; }
template <typename T>
__device__ __forceinline__ T PUe(const Ctx<T>& c, int j, int i) {
  return T(0.5) * (P2(c, j, i) + P2(c, j, wrp(i + 1, c.g.nx)));
}
template <typename T>
__device__ __forceinline__ T PVe(const Ctx<T>& c, int jv, int i) {
  return T(0.5) * (P2(c, jv, i) + P2(c, jv + 1, i));
}
template <typename T>
__device__ __forceinline__ T ue(const Ctx<T>& c, int j, int k, int i) {   // u = U / P^U, 0 on pole rows
  const GeoDev& g = c.g;
  if (j <= 0 || j >= g.ny) return T(0);
  return c.U[i3<T>(g, j, k, i)] / PUe(c, j, i);
}
template <typename T>
__device__ __forceinline__ T vte(const Ctx<T>& c, int jv, int k, int i) {  // v sin(theta) on V row jv
  return Ve(c, jv, k, i) / PVe(c, jv, i) * (T)c.g.sv[jv];
}

// ------------------------------------------------------------------------------------------------
// forward recompute
// ------------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_f2d(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int j = blockIdx.y;
  const T p0 = (T)g.p0, RT0 = (T)g.RT0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.nx; i += gridDim.x * blockDim.x) {
    const T ps = psE(c, j, i);
    const size_t id = (size_t)j * g.nx + i;
    c.s.P[id] = tsqrt<T>(ps / p0);
    c.s.L[id] = tlog<T>(ps / p0);
    c.s.Q[id] = c.s.L[id] + (T)g.phis[id] / RT0;
    T dl = 0, dq = 0;
    if (j >= 1 && j < g.ny) {
      const int M = g.M[j], n = (M + 1) / 2;
      const T dx = (T)((double)M * g.a * g.s[j] * g.dlam);
      const int pa = wrp(i + n, g.nx), pb = wrp(i + 1 - n, g.nx);
      const T la = tlog<T>(psE(c, j, pa) / p0), lb = tlog<T>(psE(c, j, pb) / p0);
      dl = (la - lb) / dx;
      const T qa = la + (T)g.phis[(size_t)j * g.nx + pa] / RT0;
      const T qb = lb + (T)g.phis[(size_t)j * g.nx + pb] / RT0;
      dq = (qa - qb) / dx;
    }
    c.s.DL[id] = dl;
    c.s.DQ[id] = dq;
  }
}

// interior columns: RT', D, S, phi', sigma-dot, omega/p
template <typename T>
__global__ void __launch_bounds__(256) k_f1(Ctx<T> c) {
  const GeoDev& g = c.g;
  int tx, k0, jy;
  xcd_tile3((int)gridDim.x, 1, (int)gridDim.y, tx, k0, jy);
  const int j = c.jr0 + c.jrs * jy;
  const int i = tx * blockDim.x + threadIdx.x;
  if (i >= g.nx) return;
  const int nx = g.nx, nz = g.nz;
  const bool all = c.fwd_all;   // the advection adjoint reads only D, S and sigma-dot
  const T b = (T)g.b;
  const int M = g.M[j], n = (M + 1) / 2;
  const T dx = (T)((double)M * g.a * g.s[j] * g.dlam);
  const T dyS = (T)(g.a * g.s[j] * g.dth), dyA = (T)(g.a * g.dth);
  const T P0 = P2(c, j, i);
  const T PV0 = PVe(c, j, i), PVm = PVe(c, j - 1, i);
  const int pa = wrp(i + n - 1, nx), pb = wrp(i - n, nx), im1 = wrp(i - 1, nx);
  const T PUa = PUe(c, j, pa), PUb = PUe(c, j, pb), PU0 = PUe(c, j, i), PUm = PUe(c, j, im1);
  C H = 0, S = 0;
  // advection: u at the U point and v sin(theta) on V row j, as k_uv forms them (rows 1..ny-1)
  const T rPU2 = all ? T(0) : T(2) / (P0 + P2(c, j, wrp(i + 1, nx)));
  const T rPVs = all ? T(0) : T(1) / (T(0.5) * (P2(c, j, i) + P2(c, j + 1, i)));
  // advection with the row-fused tail: the sigma-dot transposes of the column are formed here too
  // (the adjoint of sigma-dot at each half level, then aPi, the adjoint of the divergence and the
  // column's P share), from the output adjoints and the state at this column and its western
  // neighbour, with the same arithmetic as the per-point form.  u and v sin(theta) are then stored
  // only for the rows that the per-point kernels of the polar rows read (the row-fused kernel forms
  // them itself), and S not at all.
  const bool asdm = !all && c.adt != nullptr;
  const bool keep_uv = !all && (!asdm || j <= c.pp_n + 1 || j >= g.ny - c.pp_s - 1);
  using A = T;
  const A chA = (A)c.ch;
  A qF = 0, xF = 0, qU = 0, xU = 0, qUw = 0, xUw = 0, qVm = 0, xVm = 0, qV = 0, xV = 0;   // level k-1
  const C rP2c = 1.0 / ((C)P0 * (C)P0);
  C aPi = 0, aSt = 0;   // aPi and the column sum of aS_h = -asd_h / P^2
  if (!asdm) stg(c.s.S, ihu(g, j, 0, i), T(0));
  // the level's loads, issued one level ahead of their use
  struct L1 { T F, U, V, Uw, Vm, aF, aU, aUw, aVm, aV, Ua, Ub; };
  auto load1 = [&](int k) {
    L1 l{};
    const unsigned id = i3u(g, j, k, i), idm = i3u(g, j - 1, k, i);
    if (asdm || all) l.F = ldg(c.F, id);
    if (asdm || keep_uv) l.U = ldg(c.U, id);
    l.V = ldg(c.V, id);
    l.Vm = ldg(c.V, idm);
    if (asdm) {
      const unsigned idw = i3u(g, j, k, im1);
      l.Uw = ldg(c.U, idw);
      l.aF = ldg(c.aoF, id);
      l.aU = ldg(c.aoU, id);
      l.aUw = ldg(c.aoU, idw);
      l.aVm = ldg(c.aoV, idm);
      l.aV = ldg(c.aoV, id);
    }
    l.Ua = ldg(c.U, i3u(g, j, k, pa));
    l.Ub = ldg(c.U, i3u(g, j, k, pb));
    return l;
  };
  L1 nx1 = load1(0);
  for (int k = 0; k < nz; ++k) {
    const unsigned id = i3u(g, j, k, i);
    const L1 l = nx1;
    if (k + 1 < nz) nx1 = load1(k + 1);
    if (keep_uv) {
      stg(c.s.UA, id, l.U * rPU2);
      stg(c.s.VT, id, l.V * rPVs * (T)g.sv[j]);
    }
    if (asdm) {
      const A aF = -chA * (A)l.aF, vF = l.F;
      const A aU = -chA * (A)l.aU, vU = l.U;
      const A aUw = -chA * (A)l.aUw, vUw = l.Uw;
      const A aVm = -chA * (A)l.aVm, vVm = l.Vm;
      const A aV = -chA * (A)l.aV, vV = l.V;
      if (k >= 1) {
        const A r0 = (A)c.f.r2d[k - 1], r1 = (A)c.f.r2d[k];
        A a = 0;
        a += qF * vF * r0 - aF * xF * r1;
        const A su = qU * vU * r0 - aU * xU * r1, sw = qUw * vUw * r0 - aUw * xUw * r1;
        a += A(0.5) * (su + sw);
        a += A(0.5) * (qVm * vVm * r0 - aVm * xVm * r1);
        a += A(0.5) * (qV * vV * r0 - aV * xV * r1);
        stg(c.s.ASD, ihu(g, j, k, i), (T)a);
        aPi += g.sigh[k] * (C)(T)a * rP2c;
        aSt += -(C)(T)a * rP2c;
      }
      qF = aF; xF = vF; qU = aU; xU = vU; qUw = aUw; xUw = vUw; qVm = aVm; xVm = vVm; qV = aV; xV = vV;
    }
    if (all) {
      const T RT = b * l.F / P0;
      stg(c.s.RT, id, RT);
      H += g.cl[k] * (C)RT;
    }
    const T D = (PUa * l.Ua - PUb * l.Ub) / dx + ((T)g.sv[j] * (PV0 * l.V) - (T)g.sv[j - 1] * (PVm * l.Vm)) / dyS;
    stg(c.s.D, id, D);
    S += (C)D * g.dsig[k];
    if (!asdm) stg(c.s.S, ihu(g, j, k + 1, i), (T)S);
  }
  const C Pi = S;
  C R = 0, Sk = 0;
  const C P0s = (C)P0 * (C)P0;
  T l0 = 0, l1 = 0, lm = 0, dl0 = 0, dlm = 0;
  if (all) {
    l0 = c.s.L[(size_t)j * nx + i]; l1 = c.s.L[(size_t)(j + 1) * nx + i]; lm = c.s.L[(size_t)(j - 1) * nx + i];
    dl0 = c.s.DL[(size_t)j * nx + i]; dlm = c.s.DL[(size_t)j * nx + im1];
  }
  // sigma-dot transposes, top-down: aD_l = dsig_l (aPi + sum_{h>l} aS_h), the suffix sum being the
  // column sum less the levels above; the P share sums -2 (sigma_h Pi - S_h) asd_h / P^3
  const C Pt = (C)(T)Pi, rP3 = rP2c / (C)P0;
  C pre = 0, aP = 0;
  stg(c.s.SD, ihu(g, j, 0, i), T(0));
  // the second pass's loads, one level ahead (D, R T' and the sigma-dot adjoints are this thread's
  // own stores of the first pass)
  struct L2 { T D, RT, U, Uw, V, Vm, asd; };
  auto load2 = [&](int k) {
    L2 l{};
    const unsigned id = i3u(g, j, k, i);
    l.D = ldg((const T*)c.s.D, id);
    if (all) {
      l.RT = ldg((const T*)c.s.RT, id);
      l.U = ldg(c.U, id);
      l.Uw = ldg(c.U, i3u(g, j, k, im1));
      l.V = ldg(c.V, id);
      l.Vm = ldg(c.V, i3u(g, j - 1, k, i));
    }
    if (asdm && k >= 1) l.asd = ldg((const T*)c.s.ASD, ihu(g, j, k, i));
    return l;
  };
  L2 nx2 = load2(0);
  for (int k = 0; k < nz; ++k) {
    const unsigned id = i3u(g, j, k, i);
    const L2 l = nx2;
    if (k + 1 < nz) nx2 = load2(k + 1);
    const C D = (C)l.D;
    if (all) {
      const T RT = l.RT;
      R += g.cl[k] * (C)RT;
      stg(c.s.PHI, id, (T)(H - R + g.cpk[k] * (C)RT));
      const T zon = T(0.5) * ((l.U / PU0) * dl0 + (l.Uw / PUm) * dlm);
      const T mer = T(0.5) * ((l.V / PV0) * (l1 - l0) + (l.Vm / PVm) * (l0 - lm)) / dyA;
      stg(c.s.WP, id, (T)(((C)zon + (C)mer) - (Sk + 0.5 * D * g.dsig[k]) / (g.sig[k] * P0s)));
    }
    if (asdm) {
      if (k >= 1) {
        const C a = (C)l.asd;
        pre += -a * rP2c;
        aP += -2.0 * (g.sigh[k] * Pt - (C)(T)Sk) * rP3 * a;
      }
      stg(c.s.AD, id, (T)(g.dsig[k] * (aPi + (aSt - pre))));
    }
    Sk += D * g.dsig[k];
    stg(c.s.SD, ihu(g, j, k + 1, i), (k + 1 < nz) ? (T)((g.sigh[k + 1] * Pi - Sk) / P0s) : T(0));
  }
  if (asdm) c.s.AP2[(size_t)j * nx + i] = aP;
}

// pole columns, step 1: per (pole, level) cap divergence and zonal-mean v.grad(l) (FP64, one block each)
template <typename T>
__global__ void __launch_bounds__(256) k_f1p_red(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int k = blockIdx.x, p = blockIdx.y;
  const int j = p == 0 ? 0 : g.ny;
  const int ja = p == 0 ? 1 : g.ny - 1;
  const int jv = p == 0 ? 0 : g.ny - 1;
  const int nx = g.nx, t = threadIdx.x;
  __shared__ double red[2][4];
  const T Pp = P2(c, j, 0), lp = c.s.L[(size_t)j * nx];
  C s1 = 0, s2 = 0;
  for (int i = t; i < nx; i += blockDim.x) {
    const T pv = T(0.5) * (Pp + P2(c, ja, i));
    const T vv = Ve(c, jv, k, i);
    s1 += (C)(pv * vv);
    const T la = c.s.L[(size_t)ja * nx + i];
    s2 += (C)((vv / pv) * (p == 0 ? (la - lp) : (lp - la)));
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if ((t & 63) == 0) { red[0][t >> 6] = s1; red[1][t >> 6] = s2; }
  __syncthreads();
  C S1 = 0, S2 = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { S1 += red[0][w]; S2 += red[1][w]; }
  const C sgn = p == 0 ? 1.0 : -1.0;
  const T D = (T)(sgn * g.a * g.dlam * g.sv[jv] * S1 / g.acap);
  const T vg = (T)(S2 / ((double)nx * g.a * g.dth));
  for (int i = t; i < nx; i += blockDim.x) {
    c.s.D[i3<T>(g, j, k, i)] = D;
    c.s.WP[i3<T>(g, j, k, i)] = vg;   // v.grad(l) until step 2 overwrites it with omega/p
  }
}

// pole columns, step 2: the column scans on the pole scalars (each block redoes them over the nz
// scalars, in the same order) and the values of one level, written to the whole row
template <typename T>
__global__ void __launch_bounds__(256) k_f1p(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int k = blockIdx.x, p = blockIdx.y;
  const int j = p == 0 ? 0 : g.ny;
  const int nx = g.nx, nz = g.nz, t = threadIdx.x;
  const T b = (T)g.b;
  const T Pp = P2(c, j, 0);
  __shared__ T sRT[kMaxLevels];
  __shared__ double sD[kMaxLevels];
  for (int kk = t; kk < nz; kk += blockDim.x) {
    sRT[kk] = b * (T)c.pin[p * (nz + 1) + kk] / Pp;
    sD[kk] = (C)c.s.D[i3<T>(g, j, kk, 0)];
  }
  __syncthreads();
  auto RTl = [&](int kk) -> T { return sRT[kk]; };
  auto Dl = [&](int kk) -> C { return sD[kk]; };
  C H = 0, Pi = 0;
  for (int kk = 0; kk < nz; ++kk) {
    H += g.cl[kk] * (C)RTl(kk);
    Pi += Dl(kk) * g.dsig[kk];
  }
  C R = 0, S = 0;
  for (int kk = 0; kk < k; ++kk) {
    R += g.cl[kk] * (C)RTl(kk);
    S += Dl(kk) * g.dsig[kk];
  }
  const C P0s = (C)Pp * (C)Pp;
  const T RT = RTl(k);
  R += g.cl[k] * (C)RT;
  const T PHI = (T)(H - R + g.cpk[k] * (C)RT);
  const C D = Dl(k);
  const C vg = (C)c.s.WP[i3<T>(g, j, k, 0)];
  const T WP = (T)(vg - (S + 0.5 * D * g.dsig[k]) / (g.sig[k] * P0s));
  const T Sk = (T)S;
  S += D * g.dsig[k];
  const T SDn = (k + 1 < nz) ? (T)((g.sigh[k + 1] * Pi - S) / P0s) : T(0);
  __syncthreads();   // every thread has read this level's v.grad(l) before WP is overwritten
  for (int i = t; i < nx; i += blockDim.x) {
    const size_t id = i3<T>(g, j, k, i);
    c.s.RT[id] = RT;
    c.s.PHI[id] = PHI;
    c.s.WP[id] = WP;
    c.s.S[ih<T>(g, j, k, i)] = Sk;
    c.s.SD[ih<T>(g, j, k + 1, i)] = SDn;
    if (k == 0) c.s.SD[ih<T>(g, j, 0, i)] = T(0);
    if (k == nz - 1) c.s.S[ih<T>(g, j, nz, i)] = (T)S;
  }
}

// ------------------------------------------------------------------------------------------------
// base part of the stage transpose (interior rows: identity; pole rows: spread of the row sum) and
// pole sums of the output adjoint
// ------------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_base(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int j = row_of(c, (int)blockIdx.z, (int)gridDim.z), k = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nx) return;
  const size_t id = i3<T>(g, j, k, i);
  if (j < g.ny) c.abV[id] += c.aoV[id];
  if (j >= 1 && j < g.ny) {
    c.abU[id] += c.aoU[id];
    c.abF[id] += c.aoF[id];
    if (k == 0) c.abP[(size_t)j * g.nx + i] += c.aoP[(size_t)j * g.nx + i];
  }
}

// FP64 row sums over a pole row of a scalar-point field (per level) or of p_s (slot nz).
template <typename T>
__global__ void __launch_bounds__(64) k_pole_sum(GeoDev g, const T* f3, const T* f2, double* out) {
  const int v = blockIdx.x;   // 0 .. 2*(nz+1)-1
  const int p = v / (g.nz + 1), k = v % (g.nz + 1);
  const int j = p == 0 ? 0 : g.ny;
  C s = 0;
  if (k < g.nz) {
    if (f3) s = lane_row_sum(f3 + ((size_t)j * g.nz + k) * g.nx, g.nx, threadIdx.x);
  } else if (f2) {
    s = lane_row_sum(f2 + (size_t)j * g.nx, g.nx, threadIdx.x);
  }
  s = wave_sum(s);
  if (threadIdx.x == 0) out[p * (g.nz + 1) + k] = s;
}

// The pole sums of two level fields in one launch: blocks [0, 2(nz+1)) sum fa into outa, the next
// 2(nz+1) fb into outb, each exactly as k_pole_sum does.
template <typename T>
__global__ void __launch_bounds__(64) k_pole_sum2(GeoDev g, const T* fa, double* outa, const T* fb, double* outb) {
  const int nb = 2 * (g.nz + 1);
  const bool second = (int)blockIdx.x >= nb;
  const int v = second ? (int)blockIdx.x - nb : (int)blockIdx.x;
  const T* f3 = second ? fb : fa;
  double* out = second ? outb : outa;
  const int p = v / (g.nz + 1), k = v % (g.nz + 1);
  const int j = p == 0 ? 0 : g.ny;
  C s = 0;
  if (k < g.nz) s = lane_row_sum(f3 + ((size_t)j * g.nz + k) * g.nx, g.nx, threadIdx.x);
  s = wave_sum(s);
  if (threadIdx.x == 0) out[p * (g.nz + 1) + k] = s;
}

// The pole sums of the output adjoints of Phi (per level) and p_s (slot nz) into PS_AOF, the first
// wavefront of each block summing its row as k_pole_sum does, then the base part of the pole rows'
// transpose: the block adds its sum / nx to every stored copy of its row of the base adjoint.
template <typename T>
__global__ void __launch_bounds__(256) k_pole_sum_base(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int v = blockIdx.x;   // 0 .. 2*(nz+1)-1
  const int p = v / (g.nz + 1), k = v % (g.nz + 1);
  const int j = p == 0 ? 0 : g.ny;
  __shared__ double tot;
  if (threadIdx.x < 64) {
    const T* row = k < g.nz ? c.aoF + ((size_t)j * g.nz + k) * g.nx : c.aoP + (size_t)j * g.nx;
    const C s = wave_sum(lane_row_sum(row, g.nx, threadIdx.x));
    if (threadIdx.x == 0) {
      c.s.psum[PS_AOF * 2 * (g.nz + 1) + p * (g.nz + 1) + k] = s;
      tot = s;
    }
  }
  __syncthreads();
  const T add = (T)(tot / g.nx);
  T* dst = k < g.nz ? c.abF + ((size_t)j * g.nz + k) * g.nx : c.abP + (size_t)j * g.nx;
  for (int i = threadIdx.x; i < g.nx; i += blockDim.x) dst[i] += add;
}

// ------------------------------------------------------------------------------------------------
// adaptation: first transposes (Phi and p_s tendencies, omega/p, pressure gradients, Coriolis)
// ------------------------------------------------------------------------------------------------
// The scalar part takes the point's output adjoint of Phi, omega/p, S and D as loaded by the caller.
template <typename T>
struct A1In { T aoF, wp, S, D; };

template <typename T>
__device__ __forceinline__ A1In<T> a1_load(const Ctx<T>& c, int j, int k, int i) {
  const unsigned id = i3u(c.g, j, k, i);
  return A1In<T>{ldg(c.aoF, id), ldg((const T*)c.s.WP, id), ldg((const T*)c.s.S, ihu(c.g, j, k, i)),
                 ldg((const T*)c.s.D, id)};
}

// PM: the parts as a compile-time mask (0: the context's)
template <typename T, int PM = 0>
__device__ __forceinline__ void a1_point(const Ctx<T>& c, int j, int k, int i, const A1In<T>& in, C& aWPo, C& aSKo,
                                         C& aDo) {
  const int parts = PM ? PM : c.parts;
  aWPo = aSKo = aDo = 0;
  const GeoDev& g = c.g;
  const int nx = g.nx, ny = g.ny;
  const T b = (T)g.b, kap = (T)g.kappa;
  const C ch = c.ch;
  const size_t id = i3<T>(g, j, k, i);
  // scalar point (every row; pole rows per stored copy)
  if (parts & 1) {
    const T P = P2(c, j, i);
    const T F = Fe(c, j, k, i);
    const C gF = ch * (C)in.aoF;
    const C wp = (C)in.wp;
    const C aWP = ((C)(b * P) + (C)(kap * F)) * gF;
    const C P2c = (C)P * (C)P;
    const C Sk = (C)in.S;
    const C D = (C)in.D;
    c.s.AVGL[id] = (T)aWP;
    aWPo = aWP;
    aSKo = -aWP / (g.sig[k] * P2c);
    aDo = -0.5 * g.dsig[k] * aWP / (g.sig[k] * P2c);
    c.s.AFE[id] = (T)((C)kap * wp * gF);
    c.s.AP3[id] = (T)((C)b * wp * gF + 2.0 * (Sk + 0.5 * D * g.dsig[k]) / (g.sig[k] * P2c * (C)P) * aWP);
  }
  // U point (interior rows)
  if ((parts & 2) && j >= 1 && j < ny) {
    const int M = g.M[j], n = (M + 1) / 2;
    const T dx = (T)((double)M * g.a * g.s[j] * g.dlam);
    const int ip1 = wrp(i + 1, nx);
    const C gU = ch * (C)c.aoU[id];
    const T PU = PUe(c, j, i);
    const T dphi = (c.s.PHI[i3<T>(g, j, k, wrp(i + n, nx))] - c.s.PHI[i3<T>(g, j, k, wrp(i + 1 - n, nx))]) / dx;
    const T rtx = T(0.5) * (c.s.RT[id] + c.s.RT[i3<T>(g, j, k, ip1)]);
    const C pgf = (C)dphi + g.RT0 * (C)c.s.DQ[(size_t)j * nx + i] + (C)rtx * (C)c.s.DL[(size_t)j * nx + i];
    const T VV = T(0.25) * (Ve(c, j, k, i) + Ve(c, j, k, ip1) + Ve(c, j - 1, k, i) + Ve(c, j - 1, k, ip1));
    const T u = c.U[id] / PU;
    const T fs = (T)g.f[j] + u * (T)(g.cot[j] / g.a);
    c.s.HH[id] = (T)(-(C)PU * gU);
    c.s.FU[id] = (T)((C)fs * gU);
    c.s.AUU[id] = (T)(-(C)VV * (g.cot[j] / g.a) * gU);
    c.s.APU3[id] = (T)(-pgf * gU);
  }
  // V point (V rows)
  if ((parts & 4) && j < ny) {
    const int jv = j;
    const int im1 = wrp(i - 1, nx);
    const C gV = ch * (C)c.aoV[id];
    const T PV = PVe(c, jv, i);
    const T dyA = (T)(g.a * g.dth);
    const C pgf = ((C)(c.s.PHI[i3<T>(g, jv + 1, k, i)] - c.s.PHI[id]) +
                   g.RT0 * (C)(c.s.Q[(size_t)(jv + 1) * nx + i] - c.s.Q[(size_t)jv * nx + i]) +
                   (C)(T(0.5) * (c.s.RT[id] + c.s.RT[i3<T>(g, jv + 1, k, i)])) *
                       (C)(c.s.L[(size_t)(jv + 1) * nx + i] - c.s.L[(size_t)jv * nx + i])) / (C)dyA;
    const T UU = T(0.25) * (Ue(c, jv, k, im1) + Ue(c, jv, k, i) + Ue(c, jv + 1, k, im1) + Ue(c, jv + 1, k, i));
    const T uu = T(0.25) * (ue(c, jv, k, im1) + ue(c, jv, k, i) + ue(c, jv + 1, k, im1) + ue(c, jv + 1, k, i));
    const T fs = (T)g.fv[jv] + uu * (T)(g.cotv[jv] / g.a);
    c.s.MV[id] = (T)(-(C)PV * gV / (C)dyA);
    c.s.FV[id] = (T)((C)fs * gV);
    c.s.UV[id] = (T)((C)UU * gV * (g.cotv[jv] / g.a));
    c.s.APV3[id] = (T)(-pgf * gV);
  }
}

// First adaptation transposes (Phi and p_s tendencies, omega/p, pressure gradients, Coriolis) per
// column, bottom to top, with the suffix transpose of the column prefix sums folded in:
// aD_l = (direct part) + dsig_l (aPi + sum_{k>l} aS_k), aPi = -p0 ch aoP.
template <typename T, int KB, int PM>
__global__ void k_a12(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int j = c.jr0 + c.jrs * (int)blockIdx.y;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nx) return;
  const C aPi = -g.p0 * c.ch * (C)c.aoP[(size_t)j * g.nx + i];
  const bool sc = (PM ? PM : c.parts) & 1;
  C acc = 0;
  // levels in batches of KB, top of the batch first: the scalar-point loads of a batch are all in
  // flight before its column sums
  for (int k0 = g.nz - 1; k0 >= 0; k0 -= KB) {
    // opaque column index: addresses are formed per batch rather than held as per-array
    // induction variables across the loop
    asm volatile("" : "+v"(i));
    A1In<T> in[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) in[u] = sc ? a1_load(c, j, k0 - u >= 0 ? k0 - u : 0, i) : A1In<T>{};
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int k = k0 - u;
      if (k < 0) break;
      C aWP, aSK, aD;
      a1_point<T, PM>(c, j, k, i, in[u], aWP, aSK, aD);
      if (sc) c.s.AD[i3<T>(g, j, k, i)] = (T)(aD + g.dsig[k] * (aPi + acc));
      acc += aSK;
    }
  }
}

// The first adaptation transposes without the scalar points' column sums (parts without bit 1):
// levels are independent, one thread per (column, level, row).
template <typename T>
__global__ void k_a1lev(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int j = c.jr0 + c.jrs * (int)blockIdx.z, k = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nx) return;
  C aWP, aSK, aD;
  a1_point(c, j, k, i, A1In<T>{}, aWP, aSK, aD);
}

// gathers of the adaptation transposes at scalar, U and V points
struct A3Out {
  C aphi, art, al, aq;   // scalar point: adjoints of phi', R T', l, q
  C au, aud, adl, adq;   // U point: adjoints of u and (directly) U, leaped d+l and d+q
  C avv, avd;            // V point: adjoints of v and (directly) V
};
template <typename T>
__device__ __forceinline__ void a3_point(const Ctx<T>& c, int j, int k, int i, A3Out& o) {
  const GeoDev& g = c.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const C RT0 = g.RT0;
  const C aDy = g.a * g.dth;
  const double* sVG = c.s.psum + PS_AVGL * 2 * (nz + 1);
  const size_t id = i3<T>(g, j, k, i);
  // weights of v.grad(l) seen from V row jv: cN (scalar row jv) + cS (scalar row jv+1)
  auto cvg = [&](int jv) -> C {
    const C cN = (jv >= 1) ? 0.5 * (C)c.s.AVGL[i3<T>(g, jv, k, i)] : sVG[0 * (nz + 1) + k] / nx;
    const C cS = (jv + 1 <= ny - 1) ? 0.5 * (C)c.s.AVGL[i3<T>(g, jv + 1, k, i)] : sVG[1 * (nz + 1) + k] / nx;
    return cN + cS;
  };
  auto Lr = [&](int jr) -> C { return (C)c.s.L[(size_t)jr * nx + i]; };
  // scalar point
  {
    C aPHI = 0, aRT = 0, aL = 0, aQ = 0;
    if (j >= 1 && j < ny) {
      const int M = g.M[j], n = (M + 1) / 2;
      const C dx = (C)(T)((double)M * g.a * g.s[j] * g.dlam);
      const int im1 = wrp(i - 1, nx);
      aPHI += ((C)c.s.HH[i3<T>(g, j, k, wrp(i - n, nx))] - (C)c.s.HH[i3<T>(g, j, k, wrp(i + n - 1, nx))]) / dx;
      aRT += 0.5 * ((C)c.s.HH[id] * (C)c.s.DL[(size_t)j * nx + i] +
                    (C)c.s.HH[i3<T>(g, j, k, im1)] * (C)c.s.DL[(size_t)j * nx + im1]);
    }
    if (j >= 1) {   // V row j-1 (north): phi'(j), q(j), l(j) enter with +
      const int jv = j - 1;
      const C m = (C)c.s.MV[i3<T>(g, jv, k, i)];
      aPHI += m;
      aRT += 0.5 * (Lr(jv + 1) - Lr(jv)) * m;
      const C rty = 0.5 * ((C)c.s.RT[i3<T>(g, jv, k, i)] + (C)c.s.RT[i3<T>(g, jv + 1, k, i)]);
      const C w = (C)(Ve(c, jv, k, i) / PVe(c, jv, i)) / aDy * cvg(jv);
      aL += w + rty * m;
      aQ += RT0 * m;
    }
    if (j <= ny - 1) {   // V row j (south): enter with -
      const int jv = j;
      const C m = (C)c.s.MV[i3<T>(g, jv, k, i)];
      aPHI -= m;
      aRT += 0.5 * (Lr(jv + 1) - Lr(jv)) * m;
      const C rty = 0.5 * ((C)c.s.RT[i3<T>(g, jv, k, i)] + (C)c.s.RT[i3<T>(g, jv + 1, k, i)]);
      const C w = (C)(Ve(c, jv, k, i) / PVe(c, jv, i)) / aDy * cvg(jv);
      aL -= w + rty * m;
      aQ -= RT0 * m;
    }
    o.aphi = aPHI;
    o.art = aRT;
    o.al = aL;
    o.aq = aQ;
  }
  // U point
  if (j >= 1 && j < ny) {
    const int ip1 = wrp(i + 1, nx);
    const C dl = (C)c.s.DL[(size_t)j * nx + i];
    C au = (C)c.s.AUU[id] + 0.5 * dl * ((C)c.s.AVGL[id] + (C)c.s.AVGL[i3<T>(g, j, k, ip1)]);
    au += 0.25 * ((C)c.s.UV[i3<T>(g, j - 1, k, i)] + (C)c.s.UV[i3<T>(g, j - 1, k, ip1)] +
                  (C)c.s.UV[i3<T>(g, j, k, i)] + (C)c.s.UV[i3<T>(g, j, k, ip1)]);
    const C aUd = 0.25 * ((C)c.s.FV[i3<T>(g, j - 1, k, i)] + (C)c.s.FV[i3<T>(g, j - 1, k, ip1)] +
                          (C)c.s.FV[i3<T>(g, j, k, i)] + (C)c.s.FV[i3<T>(g, j, k, ip1)]);
    const C u = (C)(c.U[id] / PUe(c, j, i));
    const C rtx = 0.5 * ((C)c.s.RT[id] + (C)c.s.RT[i3<T>(g, j, k, ip1)]);
    const C hh = (C)c.s.HH[id];
    o.au = au;
    o.aud = aUd;
    o.adl = 0.5 * u * ((C)c.s.AVGL[id] + (C)c.s.AVGL[i3<T>(g, j, k, ip1)]) + rtx * hh;
    o.adq = RT0 * hh;
  }
  // V point
  if (j < ny) {
    const int jv = j;
    const int im1 = wrp(i - 1, nx);
    o.avv = (Lr(jv + 1) - Lr(jv)) / aDy * cvg(jv);
    C aVd = 0;
    if (jv >= 1) aVd += (C)c.s.FU[i3<T>(g, jv, k, im1)] + (C)c.s.FU[i3<T>(g, jv, k, i)];
    if (jv + 1 <= ny - 1) aVd += (C)c.s.FU[i3<T>(g, jv + 1, k, im1)] + (C)c.s.FU[i3<T>(g, jv + 1, k, i)];
    o.avd = -0.25 * aVd;
  }
}

// ------------------------------------------------------------------------------------------------
// advection transposes
// ------------------------------------------------------------------------------------------------
// The advecting velocities of the linearisation state as the advection stage forms them:
// u = U * (2 / (P_i + P_{i+1})) on interior U rows (0 on the pole rows), v sin(theta) =
// V * (1 / P^V) * sin(theta) on V rows.
template <typename T>
__global__ void k_uv(Ctx<T> c) {
  const GeoDev& g = c.g;
  int tx, k, jy;
  xcd_tile3((int)gridDim.x, g.nz, (int)gridDim.z, tx, k, jy);
  const int j = c.jr0 + c.jrs * jy;   // rows jr0 + jrs * (grid row index)
  const int i = tx * blockDim.x + threadIdx.x;
  if (i >= g.nx) return;
  const unsigned id = i3u(g, j, k, i);
  T u = T(0);
  if (j >= 1 && j < g.ny) u = ldg(c.U, id) * (T(2) / (P2(c, j, i) + P2(c, j, wrp(i + 1, g.nx))));
  stg(c.s.UA, id, u);
  if (j < g.ny) stg(c.s.VT, id, ldg(c.V, id) * (T(1) / (T(0.5) * (P2(c, j, i) + P2(c, j + 1, i)))) * (T)g.sv[j]);
}

// FAST: rows 2..ny-2 at levels 1..nz-2, where every neighbour row and level exists and none is a
// pole: the pole and boundary branches fold away and the reads shared by several outputs (with
// every store at the end) are made once.
template <typename T, bool FAST>
__device__ __forceinline__ void l1_point(const Ctx<T>& c, int j, int k, int i) {
  const GeoDev& g = c.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  auto tr = [&](bool x) { return FAST || x; };    // holds on the fast path
  auto fl = [&](bool x) { return !FAST && x; };   // fails on the fast path
  // per-point arithmetic in the field precision (every output is stored in it)
  using A = T;
  const A ch = (A)c.ch;
  const double* sF = c.s.psum + PS_AOF * 2 * (nz + 1);
  const A AN = (A)(-c.ch * sF[0 * (nz + 1) + k]), AS = (A)(-c.ch * sF[1 * (nz + 1) + k]);
  const A cc = (A)(g.a * g.dlam / (2.0 * g.acap));
  auto amF = [&](int jr, int kk, int ii) -> A { return -ch * (A)ldg(c.aoF, i3u(g, jr, kk, ii)); };
  auto amU = [&](int jr, int kk, int ii) -> A { return -ch * (A)ldg(c.aoU, i3u(g, jr, kk, ii)); };
  auto amV = [&](int jv, int kk, int ii) -> A { return -ch * (A)ldg(c.aoV, i3u(g, jv, kk, ii)); };
  auto interior = [&](int jr) { return tr(jr >= 1 && jr <= ny - 1); };
  auto FeL = [&](int jr, int kk, int ii) -> A { return FAST ? (A)ldg(c.F, i3u(g, jr, kk, ii)) : (A)Fe(c, jr, kk, ii); };
  auto UeL = [&](int jr, int kk, int ii) -> A { return FAST ? (A)ldg(c.U, i3u(g, jr, kk, ii)) : (A)Ue(c, jr, kk, ii); };
  auto sd = [&](int jr, int h, int ii) -> A { return (A)ldg(c.s.SD, ihu(g, jr, h, ii)); };
  // the forward's difference factors (rounded to the field precision)
  auto rdx2 = [&](int jr) -> A { return (A)(0.5 * c.f.rdx[jr]); };
  auto rdy2 = [&](int jr) -> A { return (A)(0.5 * c.f.rdy[jr]); };
  auto rdxv2 = [&](int jv) -> A { return (A)c.f.rdxv2[jv]; };
  auto rdyv2 = [&](int jv) -> A { return (A)c.f.rdyv2[jv]; };
  auto r2d = [&](int kk) -> A { return (A)c.f.r2d[kk]; };
  auto uA = [&](int jr, int q) -> A { return tr(jr >= 1 && jr < ny) ? (A)ldg(c.s.UA, i3u(g, jr, k, q)) : A(0); };
  auto vA = [&](int jv, int kk, int ii) -> A { return (A)ldg(c.s.VT, i3u(g, jv, kk, ii)); };
  auto ub = [&](int jr, int q) -> A {   // u averaged to integer point q of U row jr
    return A(0.5) * (uA(jr, wrp_dn(q - 1, nx)) + uA(jr, q));
  };
  auto uv = [&](int jv, int q) -> A { return A(0.5) * (uA(jv, q) + uA(jv + 1, q)); };
  auto vts = [&](int js, int kk, int ii) -> A {   // v sin(theta) on scalar row js
    if (fl(js <= 0 || js >= ny)) return A(0);
    return A(0.5) * (vA(js - 1, kk, ii) + vA(js, kk, ii));
  };
  const unsigned id = i3u(g, j, k, i);
  // every output is stored at the end, so that the loads shared by several outputs are made once
  A oFE = 0, oUU = 0, oUD = 0, oVD = 0, oVV = 0, oSD = 0;

  // ---- scalar point: adjoint of Phi (pole-read copies included)
  {
    A a = 0;
    if (interior(j)) {
      const int M = g.M[j], n = (M + 1) / 2;
      const int pm = wrp_dn(i - M, nx), pp = wrp_up(i + M, nx);
      a += (amF(j, k, pm) * uA(j, wrp_up(pm + n - 1, nx)) - amF(j, k, pp) * uA(j, wrp_dn(pp - n, nx))) * rdx2(j);
    }
    if (interior(j - 1)) a += amF(j - 1, k, i) * vA(j - 1, k, i) * rdy2(j - 1);
    if (interior(j + 1)) a -= amF(j + 1, k, i) * vA(j, k, i) * rdy2(j + 1);
    if (fl(j == 1)) a += cc * vA(0, k, i) * AN;
    if (fl(j == ny - 1)) a -= cc * vA(ny - 1, k, i) * AS;
    if (tr(k >= 1)) a += amF(j, k - 1, i) * sd(j, k, i) * r2d(k - 1);
    if (tr(k + 1 < nz)) a -= amF(j, k + 1, i) * sd(j, k + 1, i) * r2d(k + 1);
    oFE = a;
  }
  // ---- U point
  if (interior(j)) {
    const int M = g.M[j], n = (M + 1) / 2;
    // adjoint of u (U point i+1/2)
    A au = 0;
    {
      const int qa = wrp_dn(i - n + 1, nx), qb = wrp_up(i + n, nx);
      au += (amF(j, k, qa) * FeL(j, k, wrp_up(qa + M, nx)) - amF(j, k, qb) * FeL(j, k, wrp_dn(qb - M, nx))) * rdx2(j);
      auto aub = [&](int q) -> A {
        const int r1 = wrp_dn(q - n, nx), r2 = wrp_up(q - 1 + n, nx);
        return (amU(j, k, r1) * UeL(j, k, wrp_up(r1 + M, nx)) - amU(j, k, r2) * UeL(j, k, wrp_dn(r2 - M, nx))) * rdx2(j);
      };
      au += A(0.5) * (aub(i) + aub(wrp_up(i + 1, nx)));
      for (int jv : {j - 1, j}) {
        const int Mv = g.Mv[jv], nv = (Mv + 1) / 2;
        const int r1 = wrp_dn(i - nv + 1, nx), r2 = wrp_up(i + nv, nx);
        const A auv = (amV(jv, k, r1) * (A)Ve(c, jv, k, wrp_up(r1 + Mv, nx)) -
                       amV(jv, k, r2) * (A)Ve(c, jv, k, wrp_dn(r2 - Mv, nx))) * rdxv2(jv);
        au += A(0.5) * auv;
      }
    }
    oUU = au;
    // direct adjoint of U
    A aU = 0;
    {
      const int pm = wrp_dn(i - M, nx), pp = wrp_up(i + M, nx);
      aU += (amU(j, k, pm) * ub(j, wrp_up(pm + n, nx)) - amU(j, k, pp) * ub(j, wrp_dn(pp + 1 - n, nx))) * rdx2(j);
      const int ip1 = wrp_up(i + 1, nx);
      if (interior(j - 1)) {
        const A vtu = A(0.5) * (vA(j - 1, k, i) + vA(j - 1, k, ip1));
        aU += amU(j - 1, k, i) * vtu * rdy2(j - 1);
      }
      if (interior(j + 1)) {
        const A vtu = A(0.5) * (vA(j, k, i) + vA(j, k, ip1));
        aU -= amU(j + 1, k, i) * vtu * rdy2(j + 1);
      }
      if (tr(k >= 1)) aU += amU(j, k - 1, i) * A(0.5) * (sd(j, k, i) + sd(j, k, ip1)) * r2d(k - 1);
      if (tr(k + 1 < nz)) aU -= amU(j, k + 1, i) * A(0.5) * (sd(j, k + 1, i) + sd(j, k + 1, ip1)) * r2d(k + 1);
    }
    oUD = aU;
  }
  // ---- V point
  if (tr(j < ny)) {
    const int jv = j;
    const int Mv = g.Mv[jv], nv = (Mv + 1) / 2;
    A aV = 0;
    {
      const int pm = wrp_dn(i - Mv, nx), pp = wrp_up(i + Mv, nx);
      aV += (amV(jv, k, pm) * uv(jv, wrp_up(pm + nv - 1, nx)) - amV(jv, k, pp) * uv(jv, wrp_dn(pp - nv, nx))) * rdxv2(jv);
      if (tr(jv >= 1)) aV += amV(jv - 1, k, i) * vts(jv, k, i) * rdyv2(jv - 1);
      if (tr(jv + 1 <= ny - 1)) aV -= amV(jv + 1, k, i) * vts(jv + 1, k, i) * rdyv2(jv + 1);
      if (tr(k >= 1)) aV += amV(jv, k - 1, i) * A(0.5) * (sd(jv, k, i) + sd(jv + 1, k, i)) * r2d(k - 1);
      if (tr(k + 1 < nz))
        aV -= amV(jv, k + 1, i) * A(0.5) * (sd(jv, k + 1, i) + sd(jv + 1, k + 1, i)) * r2d(k + 1);
    }
    oVD = aV;
    // adjoint of v sin(theta) on this V row
    A avt = 0;
    if (interior(jv)) avt += amF(jv, k, i) * FeL(jv + 1, k, i) * rdy2(jv);
    if (interior(jv + 1)) avt -= amF(jv + 1, k, i) * FeL(jv, k, i) * rdy2(jv + 1);
    if (fl(jv == 0)) avt += cc * (A)Fe(c, 1, k, i) * AN;
    if (fl(jv == ny - 1)) avt -= cc * (A)Fe(c, ny - 1, k, i) * AS;
    auto avtu = [&](int p) -> A {
      A r = 0;
      if (interior(jv)) r += amU(jv, k, p) * UeL(jv + 1, k, p) * rdy2(jv);
      if (interior(jv + 1)) r -= amU(jv + 1, k, p) * UeL(jv, k, p) * rdy2(jv + 1);
      return r;
    };
    avt += A(0.5) * (avtu(i) + avtu(wrp_dn(i - 1, nx)));
    auto avts = [&](int js) -> A {
      if (fl(js <= 0 || js >= ny)) return A(0);
      return amV(js - 1, k, i) * (A)Ve(c, js, k, i) * rdyv2(js - 1) - amV(js, k, i) * (A)Ve(c, js - 1, k, i) * rdyv2(js);
    };
    avt += A(0.5) * (avts(jv) + avts(jv + 1));
    oVV = avt * (A)g.sv[jv];
  }
  // ---- half level h = k (1..nz-1): adjoint of sigma-dot of scalar row j
  if (tr(k >= 1)) {
    const int h = k;
    A a = 0;
    a += amF(j, h - 1, i) * FeL(j, h, i) * r2d(h - 1) -
         amF(j, h, i) * FeL(j, h - 1, i) * r2d(h);
    if (interior(j)) {
      auto asdu = [&](int p) -> A {
        return amU(j, h - 1, p) * UeL(j, h, p) * r2d(h - 1) -
               amU(j, h, p) * UeL(j, h - 1, p) * r2d(h);
      };
      a += A(0.5) * (asdu(i) + asdu(wrp_dn(i - 1, nx)));
    }
    auto asdv = [&](int jv) -> A {
      return amV(jv, h - 1, i) * (A)Ve(c, jv, h, i) * r2d(h - 1) -
             amV(jv, h, i) * (A)Ve(c, jv, h - 1, i) * r2d(h);
    };
    if (tr(j >= 1)) a += A(0.5) * asdv(j - 1);
    if (tr(j <= ny - 1)) a += A(0.5) * asdv(j);
    oSD = a;
  }
  stg(c.s.AFE, id, (T)oFE);
  if (interior(j)) {
    stg(c.s.AUU, id, (T)oUU);
    stg(c.s.AUD, id, (T)oUD);
  }
  if (tr(j < ny)) {
    stg(c.s.AVD, id, (T)oVD);
    stg(c.s.AVV, id, (T)oVV);
  }
  if (tr(k >= 1)) stg(c.s.ASD, ihu(g, j, k, i), (T)oSD);
}

// Largest divisor of nz up to 8: the level blocks of the advection transposes' launch order.
__host__ __device__ constexpr int level_block(int nz) {
  for (int d = 8; d > 1; --d)
    if (nz % d == 0) return d;
  return 1;
}

template <typename T>
__global__ void k_l1(Ctx<T> c) {
  int tx, k, jy;
  xcd_tile3_kb((int)gridDim.x, c.g.nz, (int)gridDim.z, level_block(c.g.nz), tx, k, jy);
  const int j = row_of(c, jy, (int)gridDim.z);
  const int i = tx * blockDim.x + threadIdx.x;
  if (i >= c.g.nx) return;
  if (j >= 2 && j <= c.g.ny - 2 && k >= 1 && k + 1 < c.g.nz) l1_point<T, true>(c, j, k, i);
  else l1_point<T, false>(c, j, k, i);
}

// sigma-dot transposes per column: aPi, aS_h, aP; then aD_l = dsig_l (aPi + sum_{h>l} aS_h)
template <typename T>
__global__ void k_l2(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int j = c.jr0 + c.jrs * (int)blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nx) return;
  const int nz = g.nz;
  const C P = (C)P2(c, j, i), P2c = P * P;
  const C rP2 = 1.0 / P2c, rP3 = 1.0 / (P2c * P);   // the level loops only multiply
  const C Pi = (C)ldg((const T*)c.s.S, ihu(g, j, nz, i));
  C aPi = 0, aP = 0;
  for (int h = 1; h < nz; ++h) {
    const C a = (C)ldg((const T*)c.s.ASD, ihu(g, j, h, i));
    aPi += g.sigh[h] * a * rP2;
    aP += -2.0 * (g.sigh[h] * Pi - (C)ldg((const T*)c.s.S, ihu(g, j, h, i))) * rP3 * a;
  }
  C acc = 0;   // sum_{h > l} aS_h, aS_h = -asd_h / P^2
  for (int l = nz - 1; l >= 0; --l) {
    stg(c.s.AD, i3u(g, j, l, i), (T)(g.dsig[l] * (aPi + acc)));
    if (l >= 1) acc += -(C)ldg((const T*)c.s.ASD, ihu(g, j, l, i)) * rP2;
  }
  c.s.AP2[(size_t)j * g.nx + i] = aP;
}

// ------------------------------------------------------------------------------------------------
// common tail: divergence and velocity transposes into U and V, staggered-P accumulations
// ------------------------------------------------------------------------------------------------
// Divergence and velocity transposes into U and V at one point, given the adjoints of u, U (direct),
// v, V (direct) there; returns the point's staggered-P adjoint contributions.
template <typename T>
__device__ __forceinline__ void t1_point(const Ctx<T>& c, int j, int k, int i, const A3Out& o, C& aPU3, C& aPV3) {
  const GeoDev& g = c.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double* sD = c.s.psum + PS_AD * 2 * (nz + 1);
  const size_t id = i3<T>(g, j, k, i);
  aPU3 = 0;
  aPV3 = 0;
  if (j >= 1 && j < ny) {
    const int M = g.M[j], n = (M + 1) / 2;
    const C dx = (C)(T)((double)M * g.a * g.s[j] * g.dlam);
    const C aMU = ((C)c.s.AD[i3<T>(g, j, k, wrp(i - n + 1, nx))] - (C)c.s.AD[i3<T>(g, j, k, wrp(i + n, nx))]) / dx;
    const C PU = (C)PUe(c, j, i), U = (C)c.U[id];
    c.aiU[id] = (T)((C)c.aiU[id] + o.aud + o.au / PU + PU * aMU);
    aPU3 = -U / (PU * PU) * o.au + U * aMU;
  }
  if (j < ny) {
    const int jv = j;
    const C tN = (jv >= 1) ? (C)c.s.AD[i3<T>(g, jv, k, i)] / (C)(T)(g.a * g.s[jv] * g.dth)
                           : g.a * g.dlam / g.acap * sD[0 * (nz + 1) + k];
    const C tS = (jv + 1 <= ny - 1) ? (C)c.s.AD[i3<T>(g, jv + 1, k, i)] / (C)(T)(g.a * g.s[jv + 1] * g.dth)
                                    : g.a * g.dlam / g.acap * sD[1 * (nz + 1) + k];
    const C aMV = (C)(T)g.sv[jv] * (tN - tS);
    const C PV = (C)PVe(c, jv, i), V = (C)c.V[id];
    c.aiV[id] = (T)((C)c.aiV[id] + o.avd + o.avv / PV + PV * aMV);
    aPV3 = -V / (PV * PV) * o.avv + V * aMV;
  }
}

// Adaptation, per point: the gathers of the first transposes, then the divergence and velocity
// transposes into U and V; the per-point inputs of the column sums go to scratch.
template <typename T>
__global__ void k_a3t1(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int j = c.jr0 + c.jrs * (int)blockIdx.z, k = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nx) return;
  const size_t id = i3<T>(g, j, k, i);
  A3Out o{};
  a3_point(c, j, k, i, o);
  C aPU3, aPV3;
  t1_point(c, j, k, i, o, aPU3, aPV3);
  c.s.APHI[id] = (T)o.aphi;
  c.s.ART[id] = (T)o.art;
  c.s.AL3[id] = (T)o.al;
  c.s.AQ3[id] = (T)o.aq;
  if (j >= 1 && j < g.ny) {
    c.s.ADL3[id] = (T)o.adl;
    c.s.ADQ3[id] = (T)o.adq;
    c.s.APU3[id] = (T)((C)c.s.APU3[id] + aPU3);
  }
  if (j < g.ny) c.s.APV3[id] = (T)((C)c.s.APV3[id] + aPV3);
}

// The column kernels below run a column as kLG level groups of contiguous levels (block 64 x kLG:
// 64 columns, one group per y index), so that a column's latency is that of its group's levels;
// partial FP64 sums meet in LDS and are added in group order.
constexpr int kLG = 4;

template <int N>
__device__ __forceinline__ void group_sums(double (&v)[N], double (*red)[kLG][64]) {
  const int c = threadIdx.x, q = threadIdx.y;
#pragma unroll
  for (int n = 0; n < N; ++n) red[n][q][c] = v[n];
  __syncthreads();
  if (q == 0) {
#pragma unroll
    for (int n = 0; n < N; ++n) {
      double t = red[n][0][c];
      for (int r = 1; r < kLG; ++r) t += red[n][r][c];
      v[n] = t;
    }
  }
}

// Adaptation, per column: hydrostatic transpose phi' -> R T' -> (Phi, P) and the column sums of the
// 2D adjoints.  The transpose's running sum of the phi' adjoints from the top starts each level
// group at the sum over the groups above it.
template <typename T>
__global__ void __launch_bounds__(64 * kLG) k_a4(Ctx<T> c) {
  __shared__ double red[7][kLG][64];
  const GeoDev& g = c.g;
  const int j = c.jr0 + c.jrs * (int)blockIdx.y;
  const int i = blockIdx.x * 64 + threadIdx.x, q = threadIdx.y;
  const bool live = i < g.nx;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int L = (nz + kLG - 1) / kLG, k0 = min(nz, q * L), k1 = min(nz, k0 + L);
  const T b = (T)g.b;
  const bool intr = (j >= 1 && j < ny);
  // the groups' sums of the phi' adjoints, then this group's start
  C own = 0;
  if (live)
    for (int k = k0; k < k1; ++k) own += (C)c.s.APHI[i3<T>(g, j, k, i)];
  red[0][q][threadIdx.x] = own;
  __syncthreads();
  C pre = 0;
  for (int r = 0; r < q; ++r) pre += red[0][r][threadIdx.x];
  __syncthreads();
  C v[7] = {0, 0, 0, 0, 0, 0, 0};   // aP, aPU, aPV, aL, aQ, aDL, aDQ
  if (live) {
    const C P = (C)P2(c, j, i);
    const C bP = (C)b / P, bP2 = (C)b / (P * P);
    for (int k = k0; k < k1; ++k) {
      const size_t id = i3<T>(g, j, k, i);
      const C aphi = (C)c.s.APHI[id];
      const C art = (C)c.s.ART[id] + g.cl[k] * pre + g.cpk[k] * aphi;
      pre += aphi;
      const C afe = (C)c.s.AFE[id] + bP * art;
      v[0] += (C)c.s.AP3[id] - bP2 * (C)Fe(c, j, k, i) * art;
      v[3] += (C)c.s.AL3[id];
      v[4] += (C)c.s.AQ3[id];
      if (intr) {
        v[5] += (C)c.s.ADL3[id];
        v[6] += (C)c.s.ADQ3[id];
        v[1] += (C)c.s.APU3[id];
        c.aiF[id] = (T)((C)c.aiF[id] + afe);
      } else {
        c.s.AFE[id] = (T)afe;     // pole copies: aggregated later
      }
      if (j < ny) v[2] += (C)c.s.APV3[id];
    }
  }
  group_sums<7>(v, red);
  if (live && q == 0) {
    const size_t i2 = (size_t)j * nx + i;
    c.s.AP2[i2] = v[0];
    c.s.APU2[i2] = v[1];
    c.s.APV2[i2] = v[2];
    c.s.AL2[i2] = v[3];
    c.s.AQ2[i2] = v[4];
    c.s.ADL2[i2] = v[5];
    c.s.ADQ2[i2] = v[6];
  }
}

// Advection, per column: the divergence and velocity transposes into U and V (the adjoints of u, U,
// v, V at each point come from the advection transposes) and the column sums of the staggered-P
// adjoints.
template <typename T>
__global__ void __launch_bounds__(64 * kLG) k_l3(Ctx<T> c) {
  __shared__ double red[2][kLG][64];
  const GeoDev& g = c.g;
  const int j = row_of(c, (int)blockIdx.y, (int)gridDim.y);
  const int i = blockIdx.x * 64 + threadIdx.x, q = threadIdx.y;
  const bool live = i < g.nx;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int L = (nz + kLG - 1) / kLG, k0 = min(nz, q * L), k1 = min(nz, k0 + L);
  const double* sD = c.s.psum + PS_AD * 2 * (nz + 1);
  const bool intr = (j >= 1 && j < ny);
  C v[2] = {0, 0};   // aPU, aPV
  if (live) {
    // U-point constants (as reciprocals: the level loop only multiplies)
    int n = 1;
    C rdxU = 1, PU = 1, rPU = 1;
    if (intr) {
      const int M = g.M[j];
      n = (M + 1) / 2;
      rdxU = 1.0 / (C)(T)((double)M * g.a * g.s[j] * g.dlam);
      PU = (C)PUe(c, j, i);
      rPU = 1.0 / PU;
    }
    // V-point constants
    C PV = 1, rPV = 1, rdyN = 1, rdyS = 1, capD = g.a * g.dlam / g.acap;
    if (j < ny) {
      PV = (C)PVe(c, j, i);
      rPV = 1.0 / PV;
      if (j >= 1) rdyN = 1.0 / (C)(T)(g.a * g.s[j] * g.dth);
      if (j + 1 <= ny - 1) rdyS = 1.0 / (C)(T)(g.a * g.s[j + 1] * g.dth);
    }
    const C svj = j < ny ? (C)(T)g.sv[j] : 0.0;
    const int ia = wrp(i - n + 1, nx), ib = wrp(i + n, nx);
    for (int k = k0; k < k1; ++k) {
      const unsigned id = i3u(g, j, k, i);
      A3Out o{};
      if (intr) { o.au = (C)ldg(c.s.AUU, id); o.aud = (C)ldg(c.s.AUD, id); }
      if (j < ny) { o.avv = (C)ldg(c.s.AVV, id); o.avd = (C)ldg(c.s.AVD, id); }
      if (intr) {
        const C aMU = ((C)ldg(c.s.AD, i3u(g, j, k, ia)) - (C)ldg(c.s.AD, i3u(g, j, k, ib))) * rdxU;
        const C U = (C)ldg(c.U, id);
        const C bU = c.base_in_tail ? (C)ldg(c.aoU, id) : 0.0;
        stg(c.aiU, id, (T)((C)ldg((const T*)c.aiU, id) + bU + o.aud + o.au * rPU + PU * aMU));
        v[0] += -U * (rPU * rPU) * o.au + U * aMU;
      }
      if (j < ny) {
        const int jv = j;
        const C tN = (jv >= 1) ? (C)ldg(c.s.AD, i3u(g, jv, k, i)) * rdyN : capD * sD[0 * (nz + 1) + k];
        const C tS = (jv + 1 <= ny - 1) ? (C)ldg(c.s.AD, i3u(g, jv + 1, k, i)) * rdyS : capD * sD[1 * (nz + 1) + k];
        const C aMV = svj * (tN - tS);
        const C V = (C)ldg(c.V, id);
        const C bV = c.base_in_tail ? (C)ldg(c.aoV, id) : 0.0;
        stg(c.aiV, id, (T)((C)ldg((const T*)c.aiV, id) + bV + o.avd + o.avv * rPV + PV * aMV));
        v[1] += -V * (rPV * rPV) * o.avv + V * aMV;
      }
      if (intr) stg(c.aiF, id, (T)((C)ldg((const T*)c.aiF, id) + (c.base_in_tail ? (C)ldg(c.aoF, id) : 0.0) +
                                   (C)ldg(c.s.AFE, id)));
      // (pole rows: the pole-copy adjoints stay in AFE, aggregated later)
    }
  }
  group_sums<2>(v, red);
  if (live && q == 0) {
    const size_t i2 = (size_t)j * nx + i;
    c.s.APU2[i2] = v[0];
    c.s.APV2[i2] = v[1];
    c.s.AL2[i2] = 0;
    c.s.AQ2[i2] = 0;
    c.s.ADL2[i2] = 0;
    c.s.ADQ2[i2] = 0;
  }
}

// 2D: staggered P, the leaped d+ transposes for l and q, then p_s (rows jr0 + jrs * blockIdx.y)
template <typename T>
__global__ void k_t3(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int j = c.jr0 + c.jrs * (int)blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nx) return;
  const int nx = g.nx, ny = g.ny;
  const size_t i2 = (size_t)j * nx + i;
  const int im1 = wrp(i - 1, nx);
  C aP = c.s.AP2[i2];
  if (j >= 1 && j < ny) aP += 0.5 * (c.s.APU2[i2] + c.s.APU2[(size_t)j * nx + im1]);
  if (j <= ny - 1) aP += 0.5 * c.s.APV2[i2];
  if (j >= 1) aP += 0.5 * c.s.APV2[(size_t)(j - 1) * nx + i];
  C aQ = c.s.AQ2[i2];
  C aL = c.s.AL2[i2];
  if (j >= 1 && j < ny) {
    const int M = g.M[j], n = (M + 1) / 2;
    const C dx = (C)(T)((double)M * g.a * g.s[j] * g.dlam);
    const int ra = wrp(i - n, nx), rb = wrp(i + n - 1, nx);
    aQ += (c.s.ADQ2[(size_t)j * nx + ra] - c.s.ADQ2[(size_t)j * nx + rb]) / dx;
    aL += (c.s.ADL2[(size_t)j * nx + ra] - c.s.ADL2[(size_t)j * nx + rb]) / dx;
  }
  aL += aQ;
  const C Pv = (C)P2(c, j, i);
  const C ps = (C)psE(c, j, i);
  const C aps = aP / (2.0 * g.p0 * Pv) + aL / ps;
  if (j >= 1 && j < ny) c.aiP[i2] = (T)((C)c.aiP[i2] + (c.base_in_tail ? (C)c.aoP[i2] : 0.0) + aps);
  else c.s.APSR[i2] = aps;
}

// Transpose of the p_s diffusion kappa* D_sa (eq. 1, p_s line) of an adaptation stage, FP64, added
// after k_t3: interior entries gather ch kappa* (D_sa^T a_out) directly into the input adjoint; the
// pole rows add their share to the pole-read sums (APSR) that k_t4 spreads.  The pole outputs enter
// through the FP64 sums of their replicated rows (PS_AOF, level nz).
template <typename T>
__global__ void k_dsa_adj(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int j = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nx) return;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const C kc = c.ch * g.kstar;
  const double* sF = c.s.psum + PS_AOF * 2 * (nz + 1);
  const C SAn = sF[0 * (nz + 1) + nz], SAs = sF[1 * (nz + 1) + nz];   // sums of a_out over the pole rows
  auto ao = [&](int jr, int ii) -> C { return (C)c.aoP[(size_t)jr * nx + ii]; };
  auto dy2 = [&](int jr) -> C { return g.a * g.a * g.s[jr] * g.dth * g.dth; };
  const C capN = g.sv[0] * g.dlam / (g.acap * g.dth), capS = g.sv[ny - 1] * g.dlam / (g.acap * g.dth);
  const size_t i2 = (size_t)j * nx + i;
  if (j >= 1 && j < ny) {
    const int M = g.M[j];
    const C dx = (C)M * g.a * g.s[j] * g.dlam;
    C a = (ao(j, wrp(i + M, nx)) - 2.0 * ao(j, i) + ao(j, wrp(i - M, nx))) / (dx * dx);
    a -= ao(j, i) * (g.sv[j] + g.sv[j - 1]) / dy2(j);
    if (j + 1 < ny) a += ao(j + 1, i) * g.sv[j] / dy2(j + 1);
    else a += SAs * capS;                 // the south cap's flux reads row ny-1
    if (j - 1 > 0) a += ao(j - 1, i) * g.sv[j - 1] / dy2(j - 1);
    else a += SAn * capN;                 // the north cap's flux reads row 1
    c.aiP[i2] = (T)((C)c.aiP[i2] + kc * a);
  } else if (j == 0) {
    c.s.APSR[i2] += kc * (ao(1, i) * g.sv[0] / dy2(1) - SAn * capN);
  } else {
    c.s.APSR[i2] += kc * (ao(ny - 1, i) * g.sv[ny - 1] / dy2(ny - 1) - SAs * capS);
  }
}

// pole rows: spread the FP64 row sums of the pole-copy adjoints over the stored row
template <typename T>
__global__ void k_t4(Ctx<T> c) {
  const GeoDev& g = c.g;
  const int p = blockIdx.y, k = blockIdx.x;   // k in 0..nz (nz = p_s)
  const int j = p == 0 ? 0 : g.ny;
  __shared__ double red[16];
  C s = 0;
  for (int i = threadIdx.x; i < g.nx; i += blockDim.x)
    s += (k < g.nz) ? (C)c.s.AFE[i3<T>(g, j, k, i)] : c.s.APSR[(size_t)j * g.nx + i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  C tot = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w];
  const T add = (T)(tot / g.nx);
  for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
    if (k < g.nz) c.aiF[i3<T>(g, j, k, i)] += add;
    else c.aiP[(size_t)j * g.nx + i] += add;
  }
}

// ------------------------------------------------------------------------------------------------
// Advection-stage adjoint, row-fused and tiled (interior rows whose halos fit 256 threads with 32
// owned columns; the few next to the poles on fine grids go with the pole rows through the per-point
// kernels).  The forward recompute has formed sigma-dot and, per column, the sigma-dot transposes
// down to the adjoint of the divergence (AD).  One workgroup per work item (row j, a zonal tile of w
// owned columns and a halo of hl = max(M_j, Mv_j, nv_{j-1}) columns on each side: the reach of the
// leaped advection transposes, whose centred differences span 2 M; one column per thread) walks the
// levels top to bottom.  Per level every slot stages the output adjoints of Phi, U and V rows j-1/2,
// j+1/2 (times -ch), the state they multiply, u of U rows j and j+1 (formed here from U and P, as
// the per-point kernels store it) and AD of row j in LDS; the owned columns then
// gather the transposes of every advection term that reads their Phi, U and V points (zonal leap
// offsets from LDS, the meridional and vertical neighbours from global memory, with the per-point
// form's arithmetic and order), and apply the divergence and velocity transposes into U and V with
// the column sums of the staggered-P adjoints, as the per-point column tail does.  Level rows are
// double-buffered (one barrier per level); the next level's slot values are fetched while the
// current one is computed.
// ------------------------------------------------------------------------------------------------
constexpr int kAdtLev = 11;   // per-level LDS rows (odd: consecutive slots stride an odd word count)
__host__ __device__ constexpr size_t adt_lds(int block, int elem) { return (size_t)2 * kAdtLev * block * elem; }

template <typename T>
struct AdtLev { T aF, F, aU, U, aVm, Vm, aV, V, U1, AD; };

template <typename T>
__global__ void __launch_bounds__(256) k_adt(Ctx<T> c) {
  extern __shared__ __align__(16) unsigned char smem[];
  const AatItem it = c.adt[blockIdx.x];
  if (it.j < 0) return;
  const GeoDev& g = c.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int j = it.j, hl = it.hl, w = it.w;
  const int NS = w + 2 * hl;                 // slots of the tile, halo included
  const int sl = threadIdx.x;                // this thread's slot
  const bool act = sl < NS;                  // slots past NS only meet the barriers
  const bool own = sl >= hl && sl < hl + w;  // owned column: the gathers and every global write
  int col = (it.i0 - hl + sl) % nx;
  if (col < 0) col += nx;
  const unsigned ui = (unsigned)col, uim = (unsigned)(col == 0 ? nx - 1 : col - 1);
  const unsigned uip = (unsigned)(col == nx - 1 ? 0 : col + 1);
  T* lb0 = reinterpret_cast<T*>(smem);
  T* lb1 = lb0 + kAdtLev * blockDim.x;
  enum { LaF, LF, LaU, LU, LaVm, LVm, LaV, LV, LuA, LuA1, LAD };
  using A = T;
  const bool nIn = j >= 2;            // scalar/U row j-1 is interior
  const bool sIn = j + 1 <= ny - 1;   // scalar/U row j+1 is interior
  const bool sPole = j + 1 == ny;
  const A ch = (A)c.ch;
  const int M = g.M[j], n = (M + 1) / 2;
  const int Mv = g.Mv[j], nv = (Mv + 1) / 2;
  const int nvm = (g.Mv[j - 1] + 1) / 2;
  // the forward's difference factors (rounded to the field precision)
  const A rdx2j = (A)(0.5 * c.f.rdx[j]), rdy2j = (A)(0.5 * c.f.rdy[j]);
  const A rdy2m = nIn ? (A)(0.5 * c.f.rdy[j - 1]) : A(0), rdy2p = sIn ? (A)(0.5 * c.f.rdy[j + 1]) : A(0);
  const A rdxv2m = (A)c.f.rdxv2[j - 1], rdxv2j = (A)c.f.rdxv2[j];
  const A rdyv2m = (A)c.f.rdyv2[j - 1], rdyv2j = (A)c.f.rdyv2[j], rdyv2p = sIn ? (A)c.f.rdyv2[j + 1] : A(0);
  const A cc = (A)(g.a * g.dlam / (2.0 * g.acap));
  const A svA = (A)g.sv[j];
  const double* sF = c.s.psum + PS_AOF * 2 * (nz + 1);
  const double* sD = c.s.psum + PS_AD * 2 * (nz + 1);
  // column tail constants (FP64; reciprocals: the level loop only multiplies)
  const C rdxU = 1.0 / (C)(T)((double)M * g.a * g.s[j] * g.dlam);
  const C rdyN = 1.0 / (C)(T)(g.a * g.s[j] * g.dth);
  const C rdyS = sIn ? 1.0 / (C)(T)(g.a * g.s[j + 1] * g.dth) : 1.0;
  const C capD = g.a * g.dlam / g.acap;
  const C svj = (C)(T)g.sv[j];
  const unsigned row3 = (unsigned)(nz * nx), rowh = (unsigned)((nz + 1) * nx);
  const unsigned oJ = (unsigned)j * row3, oJm = oJ - row3, oJ1 = oJ + row3;
  const unsigned ohJ = (unsigned)j * rowh, ohJ1 = ohJ + rowh;
  // 2D factors: 1 / P^U of U rows j and j+1 at this slot (u = U / P^U, as the per-point kernels store
  // it); for the owned columns 1 / P^V of V rows j-1/2 .. j+3/2 here and east (v sin(theta)) and the
  // tail's P^U, P^V
  T ruj = 0, ru1 = 0;
  T rvm = 0, rvmE = 0, rv0 = 0, rv0E = 0, rv1 = 0;
  C PU = 1, rPU = 1, PV = 1, rPV = 1;
  if (act) {
    const unsigned r0 = (unsigned)j * (unsigned)nx;
    const T P0 = ldg(c.s.P, r0 + ui), P0p = ldg(c.s.P, r0 + uip);
    const T P1 = ldg(c.s.P, r0 + nx + ui), P1p = ldg(c.s.P, r0 + nx + uip);
    ruj = T(2) / (P0 + P0p);
    if (!sPole) ru1 = T(2) / (P1 + P1p);
    if (own) {
      const T Pm = ldg(c.s.P, r0 - nx + ui), Pmp = ldg(c.s.P, r0 - nx + uip);
      rvm = T(1) / (T(0.5) * (Pm + P0));
      rvmE = T(1) / (T(0.5) * (Pmp + P0p));
      rv0 = T(1) / (T(0.5) * (P0 + P1));
      rv0E = T(1) / (T(0.5) * (P0p + P1p));
      if (sIn) rv1 = T(1) / (T(0.5) * (P1 + ldg(c.s.P, r0 + 2 * nx + ui)));
      PU = (C)(T(0.5) * (P0 + P0p));
      rPU = 1.0 / PU;
      PV = (C)(T(0.5) * (P0 + P1));
      rPV = 1.0 / PV;
    }
  }
  const T svm = (T)g.sv[j - 1], sv0 = (T)g.sv[j], sv1 = sIn ? (T)g.sv[j + 1] : T(0);
  auto load_lev = [&](int k, AdtLev<T>& v) {
    const unsigned lv = (unsigned)(k * nx) + ui;
    v.aF = ldg(c.aoF, oJ + lv);
    v.F = ldg(c.F, oJ + lv);
    v.aU = ldg(c.aoU, oJ + lv);
    v.U = ldg(c.U, oJ + lv);
    v.aVm = ldg(c.aoV, oJm + lv);
    v.Vm = ldg(c.V, oJm + lv);
    v.aV = ldg(c.aoV, oJ + lv);
    v.V = ldg(c.V, oJ + lv);
    v.U1 = sPole ? T(0) : ldg(c.U, oJ1 + lv);
    v.AD = ldg(c.s.AD, oJ + lv);
  };
  AdtLev<T> cur{}, nxt{};
  if (act) load_lev(0, cur);
  const bool bsep = c.abU != nullptr && !c.base_in_tail;   // a separate base accumulator
  A pF = 0, pU = 0, pV = 0;        // owned column: -ch a_out of Phi, U, V (row j) at level k-1
  T sdk = 0, sdkp = 0, sd1k = 0;   // sigma-dot at half level k: this column, its east neighbour, row j+1
  C aPU = 0, aPV = 0;
#pragma unroll 1
  for (int k = 0; k < nz; ++k) {
    T* L = (k & 1) ? lb1 : lb0;
    const unsigned lv = (unsigned)(k * nx);
    if (act && k + 1 < nz) load_lev(k + 1, nxt);
    // owned column: the meridional neighbours, sigma-dot at half level k+1, the accumulators
    T aFm = 0, aUm = 0, aFp = 0, Fp = 0, aUp = 0, aUpw = 0, Up = 0, Upw = 0, aVp = 0, Vp = 0;
    T ADp = 0, sdn = 0, sdnp = 0, sd1n = 0;
    T aiU0 = 0, aiV0 = 0, aiF0 = 0, abU0 = 0, abV0 = 0, abF0 = 0;
    if (own) {
      const unsigned o = oJ + lv + ui, ow = oJ + lv + uim, op = oJ + lv + uip;
      if (nIn) {
        aFm = ldg(c.aoF, o - row3);
        aUm = ldg(c.aoU, o - row3);
      }
      Fp = sPole ? (T)c.pin[(nz + 1) + k] : ldg(c.F, o + row3);
      if (sIn) {
        aFp = ldg(c.aoF, o + row3);
        aUp = ldg(c.aoU, o + row3);
        aUpw = ldg(c.aoU, ow + row3);
        Up = ldg(c.U, o + row3);
        Upw = ldg(c.U, ow + row3);
        aVp = ldg(c.aoV, o + row3);
        Vp = ldg(c.V, o + row3);
        ADp = ldg(c.s.AD, o + row3);
      }
      (void)op;
      if (k + 1 < nz) {
        const unsigned h = (unsigned)((k + 1) * nx);
        sdn = ldg(c.s.SD, ohJ + h + ui);
        sdnp = ldg(c.s.SD, ohJ + h + uip);
        sd1n = ldg(c.s.SD, ohJ1 + h + ui);
      }
      if (!c.ai_zero) {
        aiU0 = ldg(c.aiU, o);
        aiV0 = ldg(c.aiV, o);
        aiF0 = ldg(c.aiF, o);
      }
      if (bsep) {
        abU0 = ldg((const T*)c.abU, o);
        abV0 = ldg((const T*)c.abV, o);
        abF0 = ldg((const T*)c.abF, o);
      }
    }
    if (act) {
      T* q = L + sl * kAdtLev;
      q[LaF] = -ch * (A)cur.aF;
      q[LF] = cur.F;
      q[LaU] = -ch * (A)cur.aU;
      q[LU] = cur.U;
      q[LaVm] = -ch * (A)cur.aVm;
      q[LVm] = cur.Vm;
      q[LaV] = -ch * (A)cur.aV;
      q[LV] = cur.V;
      q[LuA] = cur.U * ruj;
      q[LuA1] = cur.U1 * ru1;
      q[LAD] = cur.AD;
    }
    __syncthreads();
    if (own) {
      auto R = [&](int row, int s) -> A { return (A)L[s * kAdtLev + row]; };
      const int s = sl;
      const A aF0 = R(LaF, s), aU0 = R(LaU, s), aVm0 = R(LaVm, s), aV0 = R(LaV, s);
      const A F0 = cur.F, U0 = cur.U, Vm0 = cur.Vm, V0 = cur.V;
      // v sin(theta) on V rows j-1/2 (here and east), j+1/2 (here and east), j+3/2
      const T vAm = cur.Vm * rvm * svm, vAmp = L[(s + 1) * kAdtLev + LVm] * rvmE * svm;
      const T vA0 = cur.V * rv0 * sv0, vA0p = L[(s + 1) * kAdtLev + LV] * rv0E * sv0;
      const T vAp = Vp * rv1 * sv1;
      const bool up = k >= 1, dn = k + 1 < nz;
      const A nF = dn ? -ch * (A)nxt.aF : A(0), nU = dn ? -ch * (A)nxt.aU : A(0), nV = dn ? -ch * (A)nxt.aV : A(0);
      const A r2m = up ? (A)c.f.r2d[k - 1] : A(0), r2p = dn ? (A)c.f.r2d[k + 1] : A(0);
      const A AN = (A)(-c.ch * sF[0 * (nz + 1) + k]), AS = (A)(-c.ch * sF[1 * (nz + 1) + k]);
      // ---- scalar point: adjoint of Phi
      A aFE = (R(LaF, s - M) * R(LuA, s - n) - R(LaF, s + M) * R(LuA, s + n - 1)) * rdx2j;
      if (nIn) aFE += (-ch * (A)aFm) * (A)vAm * rdy2m;
      if (sIn) aFE -= (-ch * (A)aFp) * (A)vA0 * rdy2p;
      if (j == 1) aFE += cc * (A)vAm * AN;
      if (j == ny - 1) aFE -= cc * (A)vA0 * AS;
      if (up) aFE += pF * (A)sdk * r2m;
      if (dn) aFE -= nF * (A)sdn * r2p;
      // ---- U point: adjoint of u
      A au = (R(LaF, s - n + 1) * R(LF, s + n) - R(LaF, s + n) * R(LF, s - n + 1)) * rdx2j;
      {
        auto aub = [&](int q) -> A {
          return (R(LaU, q - n) * R(LU, q + n - 1) - R(LaU, q + n - 1) * R(LU, q - n)) * rdx2j;
        };
        au += A(0.5) * (aub(s) + aub(s + 1));
        const A auvm = (R(LaVm, s - nvm + 1) * R(LVm, s + nvm) - R(LaVm, s + nvm) * R(LVm, s - nvm + 1)) * rdxv2m;
        au += A(0.5) * auvm;
        const A auvj = (R(LaV, s - nv + 1) * R(LV, s + nv) - R(LaV, s + nv) * R(LV, s - nv + 1)) * rdxv2j;
        au += A(0.5) * auvj;
      }
      // direct adjoint of U
      A aUd;
      {
        auto ub = [&](int q) -> A { return A(0.5) * (R(LuA, q - 1) + R(LuA, q)); };
        aUd = (R(LaU, s - M) * ub(s - n + 1) - R(LaU, s + M) * ub(s + n)) * rdx2j;
        if (nIn) aUd += (-ch * (A)aUm) * (A(0.5) * ((A)vAm + (A)vAmp)) * rdy2m;
        if (sIn) aUd -= (-ch * (A)aUp) * (A(0.5) * ((A)vA0 + (A)vA0p)) * rdy2p;
        if (up) aUd += pU * (A(0.5) * ((A)sdk + (A)sdkp)) * r2m;
        if (dn) aUd -= nU * (A(0.5) * ((A)sdn + (A)sdnp)) * r2p;
      }
      // ---- V point (row j+1/2): direct adjoint of V
      A aVd;
      {
        auto uv = [&](int q) -> A { return A(0.5) * (R(LuA, q) + R(LuA1, q)); };
        aVd = (R(LaV, s - Mv) * uv(s - nv) - R(LaV, s + Mv) * uv(s + nv - 1)) * rdxv2j;
        aVd += aVm0 * (A(0.5) * ((A)vAm + (A)vA0)) * rdyv2m;
        if (sIn) aVd -= (-ch * (A)aVp) * (A(0.5) * ((A)vA0 + (A)vAp)) * rdyv2p;
        if (up) aVd += pV * (A(0.5) * ((A)sdk + (A)sd1k)) * r2m;
        if (dn) aVd -= nV * (A(0.5) * ((A)sdn + (A)sd1n)) * r2p;
      }
      // adjoint of v sin(theta) on this V row
      A avt = aF0 * (A)Fp * rdy2j;
      if (sIn) avt -= (-ch * (A)aFp) * F0 * rdy2p;
      if (j == ny - 1) avt -= cc * F0 * AS;
      {
        auto avtu = [&](A aUj, A Uj, A aUn, A Un) -> A {
          A r = 0;
          r += aUj * Un * rdy2j;
          if (sIn) r -= aUn * Uj * rdy2p;
          return r;
        };
        avt += A(0.5) * (avtu(aU0, U0, -ch * (A)aUp, (A)Up) + avtu(R(LaU, s - 1), R(LU, s - 1), -ch * (A)aUpw, (A)Upw));
        const A avs0 = aVm0 * V0 * rdyv2m - aV0 * Vm0 * rdyv2j;
        const A avs1 = sIn ? aV0 * (A)Vp * rdyv2j - (-ch * (A)aVp) * V0 * rdyv2p : A(0);
        avt += A(0.5) * (avs0 + avs1);
      }
      const A aVV = avt * svA;
      // ---- divergence and velocity transposes into U and V, column sums (the per-point tail)
      const unsigned o = oJ + lv + ui;
      const bool bt = c.base_in_tail;
      const C aMU = ((C)R(LAD, s - n + 1) - (C)R(LAD, s + n)) * rdxU;
      const C Uc = (C)U0;
      stg(c.aiU, o, (T)((C)aiU0 + (bt ? (C)cur.aU : 0.0) + (C)aUd + (C)au * rPU + PU * aMU));
      aPU += -Uc * (rPU * rPU) * (C)au + Uc * aMU;
      const C tN = (C)cur.AD * rdyN;
      const C tS = sIn ? (C)ADp * rdyS : capD * sD[1 * (nz + 1) + k];
      const C aMV = svj * (tN - tS);
      const C Vc = (C)V0;
      stg(c.aiV, o, (T)((C)aiV0 + (bt ? (C)cur.aV : 0.0) + (C)aVd + (C)aVV * rPV + PV * aMV));
      aPV += -Vc * (rPV * rPV) * (C)aVV + Vc * aMV;
      stg(c.aiF, o, (T)((C)aiF0 + (bt ? (C)cur.aF : 0.0) + (C)aFE));
      if (bsep) {   // the base transpose (identity) into a separate accumulator
        stg(c.abU, o, abU0 + cur.aU);
        stg(c.abV, o, abV0 + cur.aV);
        stg(c.abF, o, abF0 + cur.aF);
        if (k == 0) {
          const unsigned o2 = (unsigned)j * (unsigned)nx + ui;
          stg(c.abP, o2, ldg((const T*)c.abP, o2) + ldg(c.aoP, o2));
        }
      }
      pF = aF0;
      pU = aU0;
      pV = aV0;
    }
    sdk = sdn;
    sdkp = sdnp;
    sd1k = sd1n;
    cur = nxt;
    // no second barrier: the next level's slot rows go to the other buffer, and the level after that
    // writes this one only past the next barrier, which every wave reaches after these gathers
  }
  if (own) {
    const size_t i2 = (size_t)j * nx + col;
    c.s.APU2[i2] = aPU;
    c.s.APV2[i2] = aPV;
    c.s.AL2[i2] = 0;
    c.s.AQ2[i2] = 0;
    c.s.ADL2[i2] = 0;
    c.s.ADQ2[i2] = 0;
  }
}

// ------------------------------------------------------------------------------------------------
// Adaptation-stage adjoint, row-fused and tiled (interior rows 1..ny-1).  One workgroup per work
// item (row j, a zonal tile of w owned columns and a halo of hl = n_j + 1 columns on each side; one
// column per thread) walks the levels top to bottom, as the forward stage kernel does: the forward
// column diagnostics of rows j and j+1 (R T', phi', D, S, omega/p) are recomputed on the way, and
// the first transposes of every output that reads row j's inputs (U row j, V rows j-1/2 and j+1/2,
// scalar rows j-1..j+1) are formed per level for every slot of the tile and staged in LDS, so that
// the owned columns' gathers at the leap offsets (+-n_j) and at +-1 are LDS reads of slots that the
// halo covers: no modular index in LDS, and the tile's LDS and registers (161 VGPRs in FP32) leave
// room for three 256-thread workgroups per CU.  The level rows are double-buffered (one barrier per
// level).  Suffix sums (the adjoint of S, the hydrostatic totals) run top-down from column totals
// taken in a first pass.  The pole rows' share goes through the per-point kernels (restricted to the
// pole rows); this kernel writes the few row-1 and row-(ny-1) intermediates those read.  On large
// grids rows 1 and ny-1, which read the pole rows' sums, run as a launch of their own (k_aat_edge)
// after them, so that the pole rows' chain can run beside the launch of the other rows.
// ------------------------------------------------------------------------------------------------
constexpr int kAatLev = 13;   // per-level LDS rows (odd: consecutive slots stride an odd word count)
__host__ __device__ constexpr size_t aat_lds(int block, int elem) { return (size_t)2 * kAatLev * block * elem; }

// STAGE (FP32, workgroups of at most kAatStageMax threads): a level's global inputs of phase 1 are
// copied straight into LDS (global_load_lds, no registers) while the previous level's phase 2 runs,
// one field-major row per input; each thread reads back only its own column's values, so the copies
// need no barrier, and they go out after a level's barrier and are read before the next one.
constexpr int kAatStg = 23;          // staged inputs per column
constexpr int kAatStageMax = 256;    // widest staged workgroup

template <typename T, bool STAGE>
__device__ __forceinline__ void aat_tile(const Ctx<T>& c) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float gin[STAGE ? kAatStg : 1][STAGE ? kAatStageMax : 1];   // staged inputs
  const AatItem it = c.aat[blockIdx.x];
  if (it.j < 0) return;
  const GeoDev& g = c.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int j = it.j, hl = it.hl, w = it.w;
  const int NS = w + 2 * hl;                 // slots of the tile, halo included
  const int sl = threadIdx.x;                // this thread's slot
  const bool act = sl < NS;                  // slots past NS only meet the barriers
  const bool own = sl >= hl && sl < hl + w;  // owned column: phase 2 and every global write
  int col = (it.i0 - hl + sl) % nx;
  if (col < 0) col += nx;
  const int colm = col == 0 ? nx - 1 : col - 1, colp = col == nx - 1 ? 0 : col + 1;
  const unsigned ui = (unsigned)col, uim = (unsigned)colm, uip = (unsigned)colp;
  // LDS: two buffers of kAatLev rows, slot-major ((slot, row) at slot * kAatLev + row)
  T* lb0 = reinterpret_cast<T*>(smem);
  T* lb1 = lb0 + kAatLev * blockDim.x;
  enum { LHH, LAV, LFVm, LFV0, LUVm, LUV0, LFU0, LFU1, LAD, LPH, LRT, LMU, Lu };

  const bool nPole = (j - 1 == 0);        // scalar row j-1 is the north pole
  const bool sPole = (j + 1 == ny);       // scalar row j+1 is the south pole
  const T b = (T)g.b, kap = (T)g.kappa;
  const C ch = c.ch;
  const int M = g.M[j], n = (M + 1) / 2;
  const T dxT = (T)((double)M * g.a * g.s[j] * g.dlam);
  const T dySj = (T)(g.a * g.s[j] * g.dth);
  const C dyS1C = sPole ? 1.0 : (C)(T)(g.a * g.s[j + 1] * g.dth);
  const T dyA = (T)(g.a * g.dth);
  const T svj = (T)g.sv[j], svm = (T)g.sv[j - 1];
  const T cotj = (T)(g.cot[j] / g.a), fj = (T)g.f[j];
  const T cot1 = sPole ? T(0) : (T)(g.cot[j + 1] / g.a), f1 = sPole ? T(0) : (T)g.f[j + 1];
  const T cvm = (T)(g.cotv[j - 1] / g.a), cv0 = (T)(g.cotv[j] / g.a);
  const T fvm = (T)g.fv[j - 1], fv0 = (T)g.fv[j];
  const C capD = g.a * g.dlam / g.acap;
  const double* sDs = c.s.psum + PS_AD * 2 * (nz + 1);
  const double* sVG = c.s.psum + PS_AVGL * 2 * (nz + 1);
  const T rdxT = T(1) / dxT, rdySjT = T(1) / dySj, rdyAT = T(1) / dyA;
  const C rnx = 1.0 / (C)nx;
  // per-point transposes run in the field precision (the sums below stay FP64)
  using A = T;
  const A chA = (A)ch, RT0A = (A)g.RT0, rdxA = (A)(1.0 / (C)dxT), rdySjA = (A)(1.0 / (C)dySj);
  const A rdyS1A = (A)(1.0 / dyS1C), rdyAA = (A)(1.0 / (C)dyA), raDyA = (A)(1.0 / (g.a * g.dth));
  const A cotjA = (A)(g.cot[j] / g.a), cvmA = (A)(g.cotv[j - 1] / g.a), cv0A = (A)(g.cotv[j] / g.a);
  const unsigned row3 = (unsigned)(nz * nx);
  const unsigned oJ = (unsigned)j * row3, oJm = oJ - row3, oJ1 = oJ + row3;

  // ---- 2D values of this slot's column (and of its western neighbour) from the forward recompute
  auto p2 = [&](int jj, unsigned ii) { return ldg(c.s.P, (unsigned)jj * (unsigned)nx + ii); };
  T Pm = 0, P0 = 0, P1 = 0, rPm = 0, rP0 = 0, rP1 = 0, PU0 = 0, rU0 = 0, rU1 = 0, rUm = 0, rU0w = 0, rU1w = 0;
  T rUmw = 0, rPV0 = 0, rPVm = 0, DLc = 0, DLw = 0, DQc = 0, dL0 = 0, dLm = 0, dQ0 = 0;
  C aPij = 0, aPi1 = 0;
  if (act) {
    Pm = p2(j - 1, ui); P0 = p2(j, ui); P1 = p2(j + 1, ui);
    const T Pmp = p2(j - 1, uip), P0p = p2(j, uip), P1p = p2(j + 1, uip);
    const T Pmw = p2(j - 1, uim), P0w = p2(j, uim), P1w = p2(j + 1, uim);
    rPm = T(1) / Pm; rP0 = T(1) / P0; rP1 = T(1) / P1;
    PU0 = T(0.5) * (P0 + P0p);
    rU0 = T(1) / PU0;
    rU1 = T(1) / (T(0.5) * (P1 + P1p));
    rUm = T(1) / (T(0.5) * (Pm + Pmp));
    rU0w = T(1) / (T(0.5) * (P0w + P0));
    rU1w = T(1) / (T(0.5) * (P1w + P1));
    rUmw = T(1) / (T(0.5) * (Pmw + Pm));
    rPV0 = T(1) / (T(0.5) * (P0 + P1));
    rPVm = T(1) / (T(0.5) * (Pm + P0));
    const unsigned r0 = (unsigned)j * (unsigned)nx;
    const T Lm = ldg(c.s.L, r0 - nx + ui), L0 = ldg(c.s.L, r0 + ui), L1 = ldg(c.s.L, r0 + nx + ui);
    dLm = L0 - Lm;
    dL0 = L1 - L0;
    dQ0 = ldg(c.s.Q, r0 + nx + ui) - ldg(c.s.Q, r0 + ui);
    DLc = ldg(c.s.DL, r0 + ui);
    DLw = ldg(c.s.DL, r0 + uim);
    DQc = ldg(c.s.DQ, r0 + ui);
    aPij = -g.p0 * ch * (C)ldg(c.aoP, r0 + ui);
    if (!sPole) aPi1 = -g.p0 * ch * (C)ldg(c.aoP, r0 + nx + ui);
  }

  // ---- pass A: column totals (hydrostatic H of rows j and j+1; sum of the adjoint of S)
  C HRj = 0, HR1 = 0, Asj = 0, As1 = 0;
  if (act) {
    constexpr int KU = 6;   // levels per batch: a batch's loads are all in flight before its sums
    for (int k0 = 0; k0 < nz; k0 += KU) {
      T vF[KU], vF1[KU], vq[KU], vq1[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + u < nz ? k0 + u : nz - 1;
        const unsigned lv = (unsigned)(k * nx) + ui;
        vF[u] = ldg(c.F, oJ + lv);
        vq[u] = ldg(c.aoF, oJ + lv);
        vF1[u] = sPole ? (T)c.pin[(nz + 1) + k] : ldg(c.F, oJ1 + lv);
        vq1[u] = sPole ? T(0) : ldg(c.aoF, oJ1 + lv);
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + u;
        if (k >= nz) break;
        const C clk = g.cl[k];
        const A rsg = (A)c.f.rsig[k];
        HRj += clk * (C)(b * vF[u] * rP0);
        HR1 += clk * (C)(b * vF1[u] * rP1);
        Asj += (C)(-((b * P0 + kap * vF[u]) * (chA * vq[u])) * rsg * (rP0 * rP0));
        if (!sPole) As1 += (C)(-((b * P1 + kap * vF1[u]) * (chA * vq1[u])) * rsg * (rP1 * rP1));
      }
    }
  }

  // ---- level loop
  // aLQ: column sum of the l and q adjoints (they enter p_s only as a sum); aDLQ: of the leaped
  // d+l and d+q adjoints (the same leap transposes both)
  C Sj = 0, pre = 0, aP = 0, aPU = 0, aPV = 0, aLQ = 0, aDLQ = 0;
  enum { GaiU, GaiV, GaiF, GFm, GFj, GF1, GUj, GUjm, GUm, GUmm, GU1, GU1m, GVj, GVjp, GVm, GVmp,
         GoF, GoU, GoV, GqVm, GqFm, GqF1, GqU1 };
  // the copies of level k's inputs into the staging rows (lane l of a wavefront lands at slot w + l)
  auto issue = [&](int k) {
    if constexpr (STAGE) {
      if (!act) return;
      const unsigned lv = (unsigned)(k * nx);
      const int wb = sl & ~63;
      auto cp = [&](int f, const T* g, unsigned o) {
        // a global-space base and a 32-bit byte offset, as ldg forms its addresses
        using GP = const __attribute__((address_space(1))) char*;
        __builtin_amdgcn_global_load_lds((GP)g + o * (unsigned)sizeof(T), &gin[f][wb], 4, 0, 0);
      };
      if (!c.ai_zero && own) {
        cp(GaiU, c.aiU, oJ + lv + ui);
        cp(GaiV, c.aiV, oJ + lv + ui);
        cp(GaiF, c.aiF, oJ + lv + ui);
      }
      if (!nPole) cp(GFm, c.F, oJm + lv + ui);
      cp(GFj, c.F, oJ + lv + ui);
      if (!sPole) cp(GF1, c.F, oJ1 + lv + ui);
      cp(GUj, c.U, oJ + lv + ui);
      cp(GUjm, c.U, oJ + lv + uim);
      if (!nPole) {
        cp(GUm, c.U, oJm + lv + ui);
        cp(GUmm, c.U, oJm + lv + uim);
      }
      if (!sPole) {
        cp(GU1, c.U, oJ1 + lv + ui);
        cp(GU1m, c.U, oJ1 + lv + uim);
      }
      cp(GVj, c.V, oJ + lv + ui);
      cp(GVjp, c.V, oJ + lv + uip);
      cp(GVm, c.V, oJm + lv + ui);
      cp(GVmp, c.V, oJm + lv + uip);
      cp(GoF, c.aoF, oJ + lv + ui);
      cp(GoU, c.aoU, oJ + lv + ui);
      cp(GoV, c.aoV, oJ + lv + ui);
      cp(GqVm, c.aoV, oJm + lv + ui);
      if (!nPole) cp(GqFm, c.aoF, oJm + lv + ui);
      if (!sPole) {
        cp(GqF1, c.aoF, oJ1 + lv + ui);
        cp(GqU1, c.aoU, oJ1 + lv + ui);
      }
    }
  };
  auto S = [&](int f) -> T { return (T)gin[f][sl]; };
  issue(0);
#pragma unroll 1
  for (int k = 0; k < nz; ++k) {
    T* L = (k & 1) ? lb1 : lb0;
    auto SL = [&](int row, int slot) -> T& { return L[slot * kAatLev + row]; };
    const C clk = g.cl[k], cpk = g.cpk[k], dsg = g.dsig[k];
    const C rsgC = c.f.rsig[k];
    const A rsg = (A)rsgC, dsgA = (A)dsg;
    const unsigned lv = (unsigned)(k * nx);
    // values of the owned columns carried from phase 1 to phase 2
    T vRTm = 0, vRT1 = 0, vPH1 = 0, vFj = 0, vUj = 0, vVj = 0, vVm = 0;
    T vAVm = 0, vAV1 = 0, vAD1 = 0, vMVm = 0, vMVj = 0, voF = 0, voU = 0, voV = 0, vAUU = 0;
    T aiU0 = 0, aiV0 = 0, aiF0 = 0;
    // ---- phase 1: per-point quantities of every slot
    if (act) {
      // the level's inputs (staged: copied into LDS during the previous level's phase 2)
      auto G = [&](int f, const T* g, unsigned o) -> T {
        if constexpr (STAGE) return S(f);
        else return ldg(g, o);
      };
      if (!c.ai_zero && own) {
        aiU0 = G(GaiU, c.aiU, oJ + lv + ui);
        aiV0 = G(GaiV, c.aiV, oJ + lv + ui);
        aiF0 = G(GaiF, c.aiF, oJ + lv + ui);
      }
      const T Fm = nPole ? (T)c.pin[k] : G(GFm, c.F, oJm + lv + ui);
      const T Fj = G(GFj, c.F, oJ + lv + ui);
      const T F1 = sPole ? (T)c.pin[(nz + 1) + k] : G(GF1, c.F, oJ1 + lv + ui);
      const T Uj = G(GUj, c.U, oJ + lv + ui), Ujm = G(GUjm, c.U, oJ + lv + uim);
      const T Um = nPole ? T(0) : G(GUm, c.U, oJm + lv + ui), Umm = nPole ? T(0) : G(GUmm, c.U, oJm + lv + uim);
      const T U1 = sPole ? T(0) : G(GU1, c.U, oJ1 + lv + ui), U1m = sPole ? T(0) : G(GU1m, c.U, oJ1 + lv + uim);
      const T Vj = G(GVj, c.V, oJ + lv + ui), Vjp = G(GVjp, c.V, oJ + lv + uip);     // V row j+1/2
      const T Vm = G(GVm, c.V, oJm + lv + ui), Vmp = G(GVmp, c.V, oJm + lv + uip);   // V row j-1/2
      voF = G(GoF, c.aoF, oJ + lv + ui);
      voU = G(GoU, c.aoU, oJ + lv + ui);
      voV = G(GoV, c.aoV, oJ + lv + ui);
      const T qVm = G(GqVm, c.aoV, oJm + lv + ui);
      const T qFm = nPole ? T(0) : G(GqFm, c.aoF, oJm + lv + ui);
      const T qF1 = sPole ? T(0) : G(GqF1, c.aoF, oJ1 + lv + ui);
      const T qU1 = sPole ? T(0) : G(GqU1, c.aoU, oJ1 + lv + ui);
      // forward: R T', phi'
      const T RTm = b * Fm * rPm, RTj = b * Fj * rP0, RT1 = b * F1 * rP1;
      HRj -= clk * (C)RTj;
      HR1 -= clk * (C)RT1;
      const T PHj = (T)(HRj + cpk * (C)RTj);
      const T PH1 = (T)(HR1 + cpk * (C)RT1);
      const T uj = Uj * rU0;
      // adjoint seeds
      const A gF = chA * (A)voF, gU = chA * (A)voU, gV = chA * (A)voV, gVm = chA * (A)qVm;
      const A aWPj = ((A)(b * P0) + (A)(kap * Fj)) * gF;
      A aWPm = 0, aWP1 = 0;
      if (!nPole) aWPm = ((A)(b * Pm) + (A)(kap * Fm)) * (chA * (A)qFm);
      C AD1 = 0;
      if (!sPole) {
        aWP1 = ((A)(b * P1) + (A)(kap * F1)) * (chA * (A)qF1);
        const C aSK1 = (C)(-aWP1 * rsg * (rP1 * rP1));
        As1 -= aSK1;
        AD1 = 0.5 * dsg * aSK1 + dsg * (aPi1 + As1);
      }
      const C aSKj = (C)(-aWPj * rsg * (rP0 * rP0));
      Asj -= aSKj;
      const C ADj = 0.5 * dsg * aSKj + dsg * (aPij + Asj);
      // U row j
      const T VV = T(0.25) * (Vj + Vjp + Vm + Vmp);
      const T fs = fj + uj * cotj;
      const A HH = -(A)PU0 * gU;
      const A FUj = (A)fs * gU;
      const A AUU = -(A)VV * cotjA * gU;
      // U row j+1 (Coriolis read of V row j+1/2)
      A FU1 = 0;
      if (!sPole) FU1 = (A)(f1 + (U1 * rU1) * cot1) * (chA * (A)qU1);
      // V row j-1/2: U rows j-1 (row 0 is the pole: u = 0) and j
      A MVm, FVm, UVm;
      {
        const T ua = nPole ? T(0) : Um * rUm, uam = nPole ? T(0) : Umm * rUmw;
        const T ub = Uj * rU0, ubm = Ujm * rU0w;
        const T UU = T(0.25) * (Umm + Um + Ujm + Uj);
        const T uu = T(0.25) * (uam + ua + ubm + ub);
        MVm = -(A)(T(0.5) * (Pm + P0)) * gVm * rdyAA;
        FVm = (A)(fvm + uu * cvm) * gVm;
        UVm = (A)UU * gVm * cvmA;
      }
      // V row j+1/2: U rows j and j+1 (row ny is the pole)
      A MVj, FVj, UVj;
      {
        const T ua = Uj * rU0, uam = Ujm * rU0w;
        const T ub = sPole ? T(0) : U1 * rU1, ubm = sPole ? T(0) : U1m * rU1w;
        const T UU = T(0.25) * (Ujm + Uj + U1m + U1);
        const T uu = T(0.25) * (uam + ua + ubm + ub);
        MVj = -(A)(T(0.5) * (P0 + P1)) * gV * rdyAA;
        FVj = (A)(fv0 + uu * cv0) * gV;
        UVj = (A)UU * gV * cv0A;
      }
      SL(LHH, sl) = (T)HH;
      SL(LAV, sl) = (T)aWPj;
      SL(LFVm, sl) = (T)FVm;
      SL(LFV0, sl) = (T)FVj;
      SL(LUVm, sl) = (T)UVm;
      SL(LUV0, sl) = (T)UVj;
      SL(LFU0, sl) = (T)FUj;
      SL(LFU1, sl) = (T)FU1;
      SL(LAD, sl) = (T)ADj;
      SL(LPH, sl) = PHj;
      SL(LRT, sl) = RTj;
      SL(LMU, sl) = PU0 * Uj;
      SL(Lu, sl) = uj;
      vRTm = RTm; vRT1 = RT1; vPH1 = PH1;
      vFj = Fj; vUj = Uj; vVj = Vj; vVm = Vm;
      vAVm = (T)aWPm; vAV1 = (T)aWP1;
      vAD1 = (T)AD1;
      vMVm = (T)MVm; vMVj = (T)MVj;
      vAUU = (T)AUU;
      if (own) {
        const unsigned oj = oJ + lv + ui;
        // intermediates the pole rows' per-point kernels read
        if (j == 1) {
          stg(c.s.AVGL, oj, (T)aWPj);
          stg(c.s.FU, oj, (T)FUj);
          stg(c.s.AD, oj, (T)ADj);
          stg(c.s.PHI, oj, PHj);
          stg(c.s.RT, oj, RTj);
        }
        if (j == ny - 1) {
          stg(c.s.AVGL, oj, (T)aWPj);
          stg(c.s.MV, oj, (T)MVj);
          stg(c.s.RT, oj, RTj);
        }
        // base transpose of the interior row (identity); where the base and input adjoints are one
        // buffer, into the accumulator values already fetched for the second phase
        if (c.abU) {
          if (c.abF == c.aiF) aiF0 += voF; else stg(c.abF, oj, ldg(c.abF, oj) + voF);
          if (c.abU == c.aiU) aiU0 += voU; else stg(c.abU, oj, ldg(c.abU, oj) + voU);
          if (c.abV == c.aiV) aiV0 += voV; else stg(c.abV, oj, ldg(c.abV, oj) + voV);
          if (k == 0) {
            const unsigned o2 = (unsigned)j * (unsigned)nx + ui;
            stg(c.abP, o2, ldg(c.abP, o2) + ldg(c.aoP, o2));
          }
        }
      }
    }
    __syncthreads();
    if (k + 1 < nz) issue(k + 1);

    // ---- phase 2: forward D, S, omega/p; gathers; transposes into the owned columns
    if (own) {
      const int sm = sl - 1, sp = sl + 1;
      const unsigned oj = oJ + lv + ui;
      const T vRTj = SL(LRT, sl), vPHj = SL(LPH, sl);
      const A vAVj = (A)SL(LAV, sl), vADj = (A)SL(LAD, sl), vHH = (A)SL(LHH, sl);
      const A vUVm = (A)SL(LUVm, sl), vUVj = (A)SL(LUV0, sl), vFVm = (A)SL(LFVm, sl), vFVj = (A)SL(LFV0, sl);
      const A vFUj = (A)SL(LFU0, sl), vFU1 = (A)SL(LFU1, sl);
      const T PV0 = T(0.5) * (P0 + P1), PVm = T(0.5) * (Pm + P0);
      // forward D, S, omega/p (as the forward recompute forms them)
      const T D = (SL(LMU, sl + n - 1) - SL(LMU, sl - n)) * rdxT +
                  (svj * (PV0 * vVj) - svm * (PVm * vVm)) * rdySjT;
      const C SkC = Sj;
      Sj += (C)D * dsg;
      const T zon = T(0.5) * (SL(Lu, sl) * DLc + SL(Lu, sm) * DLw);
      const T mer = T(0.5) * ((vVj * rPV0) * dL0 + (vVm * rPVm) * dLm) * rdyAT;
      const T Sh = (T)(SkC + 0.5 * (C)D * dsg);   // S at the full level
      const A rP2A = rP0 * rP0;
      const A wp = (A)((zon + mer) - Sh * rsg * rP2A);
      const A gF = chA * (A)voF, aWP = vAVj;
      const A AFE = kap * wp * gF;
      const A AP3 = b * wp * gF + A(2) * Sh * rsg * (rP2A * rP0) * aWP;
      // U point: pressure gradient seen by U row j
      const T dphi = (SL(LPH, sl + n) - SL(LPH, sl + 1 - n)) * rdxT;
      const T rtx = T(0.5) * (vRTj + SL(LRT, sp));
      const A pgf = (A)dphi + RT0A * (A)DQc + (A)rtx * (A)DLc;
      const A gU = chA * (A)voU, gV = chA * (A)voV;
      const A APU3 = -pgf * gU;
      // V point: pressure gradient seen by V row j+1/2
      const A pgfV = ((A)(vPH1 - vPHj) + RT0A * (A)dQ0 + (A)(T(0.5) * (vRTj + vRT1)) * (A)dL0) * rdyAA;
      const A APV3 = -pgfV * gV;
      // gathers: scalar point
      const A mM = (A)vMVm, mJ = (A)vMVj;
      const A aPHI = ((A)SL(LHH, sl - n) - (A)SL(LHH, sl + n - 1)) * rdxA + mM - mJ;
      const A aRT = A(0.5) * ((A)SL(LHH, sl) * (A)DLc + (A)SL(LHH, sm) * (A)DLw) +
                    A(0.5) * (A)dLm * mM + A(0.5) * (A)dL0 * mJ;
      const A cvgm = (nPole ? (A)(sVG[0 * (nz + 1) + k] * rnx) : A(0.5) * (A)vAVm) + A(0.5) * vAVj;
      const A cvgj = A(0.5) * vAVj + (sPole ? (A)(sVG[1 * (nz + 1) + k] * rnx) : A(0.5) * (A)vAV1);
      const A rtym = A(0.5) * ((A)vRTm + (A)vRTj), rtyj = A(0.5) * ((A)vRTj + (A)vRT1);
      const A wm = (A)(vVm * rPVm) * raDyA * cvgm, wj = (A)(vVj * rPV0) * raDyA * cvgj;
      const A aL = (wm + rtym * mM) - (wj + rtyj * mJ);
      const A aQ = RT0A * mM - RT0A * mJ;
      // gathers: U point
      const A dl = (A)DLc;
      const A au = (A)vAUU + A(0.5) * dl * (vAVj + (A)SL(LAV, sp)) +
                   A(0.25) * (vUVm + (A)SL(LUVm, sp) + vUVj + (A)SL(LUV0, sp));
      const A aUd = A(0.25) * (vFVm + (A)SL(LFVm, sp) + vFVj + (A)SL(LFV0, sp));
      const A rPUc = (A)rU0;
      const A u = (A)(vUj * rU0);
      const A rtxA = A(0.5) * ((A)vRTj + (A)SL(LRT, sp));
      const A adl = A(0.5) * u * (vAVj + (A)SL(LAV, sp)) + rtxA * vHH;
      const A adq = RT0A * vHH;
      // gathers: V point
      const A avv = (A)dL0 * raDyA * cvgj;
      A aVd = (A)SL(LFU0, sm) + vFUj;
      if (!sPole) aVd += (A)SL(LFU1, sm) + vFU1;
      const A avd = A(-0.25) * aVd;
      // divergence and velocity transposes
      const A aMU = ((A)SL(LAD, sl - n + 1) - (A)SL(LAD, sl + n)) * rdxA;
      const A PUc = (A)PU0, Uc = (A)vUj;
      // (an FP32 sum rounded once equals the FP64 sum rounded to FP32: 53 >= 2 * 24 + 2 bits)
      stg(c.aiU, oj, (T)(aiU0 + (aUd + au * rPUc + PUc * aMU)));
      const A aPU3 = -Uc * (rPUc * rPUc) * au + Uc * aMU;
      const A tN = vADj * rdySjA;
      const A tS = sPole ? (A)(capD * sDs[1 * (nz + 1) + k]) : (A)vAD1 * rdyS1A;
      const A aMV = (A)svj * (tN - tS);
      const A PVc = (A)PV0, Vc = (A)vVj, rPVc = (A)rPV0;
      stg(c.aiV, oj, (T)(aiV0 + (avd + avv * rPVc + PVc * aMV)));
      const A aPV3 = -Vc * (rPVc * rPVc) * avv + Vc * aMV;
      // hydrostatic transpose and column sums
      const A art = aRT + (A)(clk * pre) + (A)cpk * aPHI;
      pre += (C)aPHI;
      const A afe = AFE + b * rP0 * art;
      aP += (C)(AP3 - b * rP2A * (A)vFj * art);
      aLQ += (C)(aL + aQ);
      aDLQ += (C)(adl + adq);
      aPU += (C)(APU3 + aPU3);
      aPV += (C)(APV3 + aPV3);
      stg(c.aiF, oj, (T)(aiF0 + afe));
    }
    (void)dsgA;
    // no second barrier: the next level's phase 1 writes the other buffer, and the level after that
    // writes this one only past the next barrier, which every wave reaches after this phase 2
  }
  if (own) {
    const size_t i2 = (size_t)j * nx + col;
    c.s.AP2[i2] = aP;
    c.s.APU2[i2] = aPU;
    c.s.APV2[i2] = aPV;
    c.s.AL2[i2] = aLQ;
    c.s.AQ2[i2] = 0;
    c.s.ADL2[i2] = aDLQ;
    c.s.ADQ2[i2] = 0;
  }
}

// The tiles of the interior rows (all of them, or rows 2..ny-2 when rows 1 and ny-1 run apart).
template <typename T>
__global__ void __launch_bounds__(kAatMaxBlock, sizeof(T) == 4 ? 3 : 2) k_aat(Ctx<T> c) {
  aat_tile<T, sizeof(T) == 4>(c);
}

// The tiles of rows 1 and ny-1, launched after the pole rows' sums that they read.
template <typename T>
__global__ void __launch_bounds__(kAatMaxBlock, sizeof(T) == 4 ? 3 : 2) k_aat_edge(Ctx<T> c) {
  aat_tile<T, sizeof(T) == 4>(c);
}

// Workgroups wider than the staging rows: the inputs are loaded at their level.
template <typename T>
__global__ void __launch_bounds__(kAatMaxBlock, sizeof(T) == 4 ? 3 : 2) k_aat_wide(Ctx<T> c) {
  aat_tile<T, false>(c);
}

// The base transpose of a stage applied in place: pole rows of Phi and p_s become the spread of
// their row mean (FP64 sum), pole rows of U become 0; interior rows and V are left as they are.
template <typename T>
__global__ void __launch_bounds__(256) k_base_inplace(GeoDev g, T* U, T* F, T* P) {
  const int p = blockIdx.y, k = blockIdx.x;   // k in 0..nz (nz = p_s)
  const int j = p == 0 ? 0 : g.ny;
  __shared__ double red[4];
  T* row = (k < g.nz) ? F + ((size_t)j * g.nz + k) * g.nx : P + (size_t)j * g.nx;
  C s = 0;
  for (int i = threadIdx.x; i < g.nx; i += blockDim.x) s += (C)row[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  C tot = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w];
  const T mean = (T)(tot / g.nx);
  for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
    row[i] = mean;
    if (k < g.nz) U[((size_t)j * g.nz + k) * g.nx + i] = T(0);
  }
}

// Dynamic LDS above 64 KB is enabled once per kernel.
template <auto Kernel>
hipError_t allow_lds_adj(size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  static bool done = false;
  if (done) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(Kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess) done = true;
  return e;
}

// The tiled row-fused adaptation adjoint serves every grid whose rows' halos leave tiles of at least
// 32 columns (the handle then holds its work items).
template <typename T>
bool aar_used(const Ctx<T>& c) {
  return c.aat != nullptr && c.aat_n > 0 && c.g.ny >= 4;
}

// rows 1 and ny-1 in a launch of their own (on the side stream when the handle has one)
template <typename T>
bool aar_split(const Ctx<T>& c) {
  return aar_used(c) && c.aat_edge_n > 0;
}

// the staged form serves FP32 workgroups up to the staging rows' width
template <typename T>
bool aat_staged(const Ctx<T>& c) {
  return sizeof(T) == 4 && c.aat_blk <= kAatStageMax;
}

template <typename T>
hipError_t launch_aar_edge(const Ctx<T>& c, hipStream_t s) {
  const size_t lds = aat_lds(c.aat_blk, (int)sizeof(T));
  const bool st = aat_staged(c);
  hipError_t e = st ? allow_lds_adj<k_aat_edge<T>>(lds) : allow_lds_adj<k_aat_wide<T>>(lds);
  if (e != hipSuccess) return e;
  Ctx<T> ce = c;
  ce.aat = c.aat + c.aat_n;
  ce.aat_n = c.aat_edge_n;
  if (st) hipLaunchKernelGGL((k_aat_edge<T>), dim3(ce.aat_n), dim3(ce.aat_blk), lds, s, ce);
  else hipLaunchKernelGGL((k_aat_wide<T>), dim3(ce.aat_n), dim3(ce.aat_blk), lds, s, ce);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_aar(const Ctx<T>& c, hipStream_t s) {
  const size_t lds = aat_lds(c.aat_blk, (int)sizeof(T));
  const bool st = aat_staged(c);
  hipError_t e = st ? allow_lds_adj<k_aat<T>>(lds) : allow_lds_adj<k_aat_wide<T>>(lds);
  if (e != hipSuccess) return e;
  KTimer* t = c.timer;
  const bool timed = t && t->armed && t->n < t->cap;
  if (timed && (e = hipEventRecord(t->ev[2 * t->n], s)) != hipSuccess) return e;
  if (st) hipLaunchKernelGGL((k_aat<T>), dim3(c.aat_n), dim3(c.aat_blk), lds, s, c);
  else hipLaunchKernelGGL((k_aat_wide<T>), dim3(c.aat_n), dim3(c.aat_blk), lds, s, c);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (timed) {
    if ((e = hipEventRecord(t->ev[2 * t->n + 1], s)) != hipSuccess) return e;
    ++t->n;
  }
  return hipSuccess;
}

// The tiled row-fused advection adjoint serves every grid whose rows' halos fit (the handle then
// holds its work items).
template <typename T>
bool adt_used(const Ctx<T>& c) {
  return c.adt != nullptr && c.adt_n > 0;
}

// With the rows next to the poles in the per-point set (pp_n, pp_s >= 1) the tiles read nothing of
// the pole rows' chain but the output adjoint's pole sums, so that chain can run on the second stream
// beside them.
template <typename T>
bool adt_fork(const Ctx<T>& c) {
  return adt_used(c) && c.side != nullptr && c.pp_n >= 1 && c.pp_s >= 1;
}

// The next stage's 2D recompute (P, l, q and the leaped d+l, d+q of its input) into the other set of
// 2D fields, launched at the end of this stage's pole-row chain: it reads only the recorded input,
// and the set it writes is free (this stage reads the other one).
template <typename T>
void launch_f2d_next(const Ctx<T>& c, hipStream_t s) {
  if (!c.next_ps) return;
  Ctx<T> cn = c;
  cn.P = c.next_ps;
  cn.pin = c.next_pin;
  cn.s.P = c.next2d[0]; cn.s.L = c.next2d[1]; cn.s.Q = c.next2d[2]; cn.s.DL = c.next2d[3]; cn.s.DQ = c.next2d[4];
  const int gx = (c.g.nx + 255) / 256;
  hipLaunchKernelGGL((k_f2d<T>), dim3(gx, c.g.ny + 1), dim3(256), 0, s, cn);
}

template <typename T>
hipError_t launch_adt(const Ctx<T>& c, hipStream_t s) {
  const size_t lds = adt_lds(c.adt_blk, (int)sizeof(T));
  hipLaunchKernelGGL((k_adt<T>), dim3(c.adt_n), dim3(c.adt_blk), lds, s, c);
  return hipGetLastError();
}

template <typename T>
hipError_t run_stage_adjoint(const Ctx<T>& c, hipStream_t s, bool adapt) {
  const GeoDev& g = c.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int tb = 256;
  const int gx = (nx + tb - 1) / tb;
  const dim3 g3(gx, nz, ny + 1), g2(gx, ny + 1), gcol_int(gx, ny - 1);
  const bool rows = adapt && aar_used(c);
  // the row-fused stage adjoints with a second stream: the work on the pole rows and the per-point
  // rows (pole-column recompute, their base transpose, the output adjoint's pole sums) opens the pole
  // rows' chain there, forked once the full-grid recompute is done; the row-fused launch that follows
  // on this stream reads none of it
  const bool fork = adapt ? rows && aar_split(c) && c.side != nullptr : adt_fork(c);
  if (!c.f2d_ready) hipLaunchKernelGGL((k_f2d<T>), g2, dim3(tb), 0, s, c);
  Ctx<T> cf = c;
  cf.jr0 = 1;
  cf.jrs = 1;
  cf.fwd_all = adapt ? 1 : 0;
  // the row-fused kernel recomputes its rows itself (and writes what the pole rows read)
  if (!rows) hipLaunchKernelGGL((k_f1<T>), gcol_int, dim3(tb), 0, s, cf);
  hipStream_t es = s;
  if (fork) {
    hipError_t e = hipEventRecord(c.side->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c.side->s, c.side->fork, 0);
    if (e != hipSuccess) return e;
    es = c.side->s;
  }
  hipLaunchKernelGGL((k_f1p_red<T>), dim3(nz, 2), dim3(256), 0, es, c);
  hipLaunchKernelGGL((k_f1p<T>), dim3(nz, 2), dim3(256), 0, es, c);
  if (c.abU && !c.base_in_tail) {
    // interior rows' base transpose is folded into the row-fused kernels (the adaptation's and the
    // advection's, for their rows) or the column tail (advection with one accumulator); V row 1/2
    // stays here for the row-fused adaptation, the per-point rows for the row-fused advection
    if (rows) {
      hipLaunchKernelGGL((k_base<T>), dim3(gx, nz, 1), dim3(tb), 0, es, c);
    } else if (!adapt && adt_used(c)) {
      Ctx<T> cw = c;
      cw.rsplit = c.pp_n + 1;
      hipLaunchKernelGGL((k_base<T>), dim3(gx, nz, c.pp_n + c.pp_s + 2), dim3(tb), 0, es, cw);
    } else {
      hipLaunchKernelGGL((k_base<T>), g3, dim3(tb), 0, es, c);
    }
  }
  if (c.abU)
    hipLaunchKernelGGL((k_pole_sum_base<T>), dim3(2 * (nz + 1)), dim3(256), 0, es, c);
  else
    hipLaunchKernelGGL((k_pole_sum<T>), dim3(2 * (nz + 1)), dim3(64), 0, es, g, c.aoF, c.aoP,
                       c.s.psum + PS_AOF * 2 * (nz + 1));
  // (process-specific part is launched by the caller between these two groups)
  return hipGetLastError();
}

template <typename T>
hipError_t run_adapt(const Ctx<T>& c, hipStream_t s) {
  const GeoDev& g = c.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int tb = 256;
  const int gx = (nx + tb - 1) / tb;
  const int gx64 = (nx + 63) / 64;   // column kernels: 64 columns x kLG level groups
  const dim3 g3(gx, nz, ny + 1), g2(gx, ny + 1);
  if (aar_used(c)) {
    // pole rows through the per-point kernels, interior rows row-fused.  With the rows split and a
    // second stream, the pole rows' chain (with rows 1 and ny-1, which read the pole rows' sums and
    // write what the pole rows' gathers read) runs there beside the other rows' launch: the two touch
    // disjoint rows of every output and scratch field, and every read-modify-write of a pole row
    // (base spread, input adjoint) is on the chain or came before the fork.
    const bool split = aar_split(c);
    const bool fork = split && c.side != nullptr;
    const hipStream_t ps = fork ? c.side->s : s;
    hipError_t e = hipSuccess;
    if (fork && (e = launch_aar<T>(c, s)) != hipSuccess) return e;
    Ctx<T> cp = c;
    cp.jr0 = 0;
    cp.jrs = ny;
    cp.parts = 1;   // scalar points of the pole rows (their sums feed the interior rows)
    hipLaunchKernelGGL((k_a12<T, 6, 1>), dim3(gx, 2), dim3(tb), 0, ps, cp);
    hipLaunchKernelGGL((k_pole_sum2<T>), dim3(4 * (nz + 1)), dim3(64), 0, ps, g, (const T*)c.s.AD,
                       c.s.psum + PS_AD * 2 * (nz + 1), (const T*)c.s.AVGL, c.s.psum + PS_AVGL * 2 * (nz + 1));
    if (!fork && (e = launch_aar<T>(c, s)) != hipSuccess) return e;
    if (split && (e = launch_aar_edge<T>(c, ps)) != hipSuccess) return e;
    Ctx<T> cv = c;   // V row 1/2: reads phi' and R T' of row 1, written by the row-fused kernel
    cv.parts = 4;
    hipLaunchKernelGGL((k_a1lev<T>), dim3(gx, nz, 1), dim3(tb), 0, ps, cv);
    cp.parts = 7;
    hipLaunchKernelGGL((k_a3t1<T>), dim3(gx, nz, 2), dim3(tb), 0, ps, cp);
    hipLaunchKernelGGL((k_a4<T>), dim3(gx64, 2), dim3(64, kLG), 0, ps, cp);
    if (fork) {
      // without D_sa the pole rows' p_s transpose and the spread of the pole-copy sums read only the
      // chain's results: they close it, and this stream takes rows 1..ny-1 of k_t3 after the join
      if (g.kstar == 0.0) {
        hipLaunchKernelGGL((k_t3<T>), dim3(gx, 2), dim3(tb), 0, ps, cp);   // rows 0 and ny
        hipLaunchKernelGGL((k_t4<T>), dim3(nz + 1, 2), dim3(256), 0, ps, c);
      }
      launch_f2d_next<T>(c, ps);
      if ((e = hipEventRecord(c.side->join, ps)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(s, c.side->join, 0)) != hipSuccess) return e;
      if (g.kstar == 0.0) {
        Ctx<T> ci = c;
        ci.jr0 = 1;
        ci.jrs = 1;
        hipLaunchKernelGGL((k_t3<T>), dim3(gx, ny - 1), dim3(tb), 0, s, ci);
        return hipGetLastError();
      }
    }
  } else {
    hipLaunchKernelGGL((k_a12<T, 1, 0>), g2, dim3(tb), 0, s, c);
    hipLaunchKernelGGL((k_pole_sum2<T>), dim3(4 * (nz + 1)), dim3(64), 0, s, g, (const T*)c.s.AD,
                       c.s.psum + PS_AD * 2 * (nz + 1), (const T*)c.s.AVGL, c.s.psum + PS_AVGL * 2 * (nz + 1));
    hipLaunchKernelGGL((k_a3t1<T>), g3, dim3(tb), 0, s, c);
    hipLaunchKernelGGL((k_a4<T>), dim3(gx64, ny + 1), dim3(64, kLG), 0, s, c);
  }
  hipLaunchKernelGGL((k_t3<T>), g2, dim3(tb), 0, s, c);
  if (g.kstar != 0.0) hipLaunchKernelGGL((k_dsa_adj<T>), g2, dim3(tb), 0, s, c);
  hipLaunchKernelGGL((k_t4<T>), dim3(nz + 1, 2), dim3(256), 0, s, c);
  return hipGetLastError();
}

template <typename T>
hipError_t run_advect(const Ctx<T>& c, hipStream_t s) {
  const GeoDev& g = c.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int tb = 256;
  const int gx = (nx + tb - 1) / tb;
  const int gx64 = (nx + 63) / 64;   // column kernels: 64 columns x kLG level groups
  const dim3 g3(gx, nz, ny + 1), g2(gx, ny + 1);
  // u and v sin(theta) of rows 1..ny-1 come from the forward recompute (k_f1); here the pole rows
  Ctx<T> cp = c;
  cp.jr0 = 0;
  cp.jrs = ny;
  if (adt_fork(c)) {
    // the tiles on the stage's stream; beside them on the second stream (forked with the pole
    // columns' recompute) the pole rows and the rows next to them through the per-point kernels: the
    // two touch disjoint rows of every output and scratch field
    const hipStream_t ps = c.side->s;
    Ctx<T> cw = c;
    cw.rsplit = c.pp_n + 1;
    const int nw = c.pp_n + c.pp_s + 2;
    hipError_t e = launch_adt<T>(c, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_uv<T>), dim3(gx, nz, 2), dim3(tb), 0, ps, cp);
    hipLaunchKernelGGL((k_l1<T>), dim3(gx, nz, nw), dim3(tb), 0, ps, cw);
    hipLaunchKernelGGL((k_l2<T>), dim3(gx, 2), dim3(tb), 0, ps, cp);
    hipLaunchKernelGGL((k_pole_sum<T>), dim3(2 * (nz + 1)), dim3(64), 0, ps, g, (const T*)c.s.AD,
                       (const T*)nullptr, c.s.psum + PS_AD * 2 * (nz + 1));
    hipLaunchKernelGGL((k_l3<T>), dim3(gx64, nw), dim3(64, kLG), 0, ps, cw);
    // the pole rows' p_s transpose and the spread of the pole-copy sums read only the chain's results
    hipLaunchKernelGGL((k_t3<T>), dim3(gx, 2), dim3(tb), 0, ps, cp);
    hipLaunchKernelGGL((k_t4<T>), dim3(nz + 1, 2), dim3(256), 0, ps, c);
    launch_f2d_next<T>(c, ps);
    if ((e = hipEventRecord(c.side->join, ps)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, c.side->join, 0)) != hipSuccess) return e;
    Ctx<T> ci = c;
    ci.jr0 = 1;
    ci.jrs = 1;
    hipLaunchKernelGGL((k_t3<T>), dim3(gx, ny - 1), dim3(tb), 0, s, ci);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_uv<T>), dim3(gx, nz, 2), dim3(tb), 0, s, cp);
  if (adt_used(c)) {
    // the pole rows and the rows next to them whose halos do not fit the tiles (rows 0..pp_n and
    // ny-pp_s..ny) through the per-point kernels; the interior rows' sigma-dot transposes came with
    // the forward recompute (k_l2 serves the pole rows), the other rows are row-fused
    Ctx<T> cw = c;
    cw.rsplit = c.pp_n + 1;
    const int nw = c.pp_n + c.pp_s + 2;
    hipLaunchKernelGGL((k_l1<T>), dim3(gx, nz, nw), dim3(tb), 0, s, cw);
    hipLaunchKernelGGL((k_l2<T>), dim3(gx, 2), dim3(tb), 0, s, cp);
    hipLaunchKernelGGL((k_pole_sum<T>), dim3(2 * (nz + 1)), dim3(64), 0, s, g, (const T*)c.s.AD,
                       (const T*)nullptr, c.s.psum + PS_AD * 2 * (nz + 1));
    const hipError_t e = launch_adt<T>(c, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_l3<T>), dim3(gx64, nw), dim3(64, kLG), 0, s, cw);
  } else {
    hipLaunchKernelGGL((k_l1<T>), g3, dim3(tb), 0, s, c);
    hipLaunchKernelGGL((k_l2<T>), g2, dim3(tb), 0, s, c);
    hipLaunchKernelGGL((k_pole_sum<T>), dim3(2 * (nz + 1)), dim3(64), 0, s, g, (const T*)c.s.AD,
                       (const T*)nullptr, c.s.psum + PS_AD * 2 * (nz + 1));
    hipLaunchKernelGGL((k_l3<T>), dim3(gx64, ny + 1), dim3(64, kLG), 0, s, c);
  }
  hipLaunchKernelGGL((k_t3<T>), g2, dim3(tb), 0, s, c);
  hipLaunchKernelGGL((k_t4<T>), dim3(nz + 1, 2), dim3(256), 0, s, c);
  return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// workspace and driver (the handle layout is private to api.hip; it exposes what we need here)
// ------------------------------------------------------------------------------------------------

namespace {

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr int kN3 = 27;   // 3D scalar-size scratch fields (4 forward + 23 adjoint)
constexpr int kNH = 3;    // half-level fields
constexpr int kN2T = 10;  // 2D T fields: two sets of P, l, q, d+l, d+q (a stage's and the next one's)
constexpr int kN2D = 8;   // 2D FP64 fields

struct Layout {
  size_t n3, nh, n2, state;
  size_t traj_off, lam_off, f3_off, fh_off, f2t_off, f2d_off, psum_off, pole_off, tpole_off, total;
};

Layout layout(const HandleView& v) {
  Layout L;
  const GeoDev& g = v.g;
  L.n3 = (size_t)(g.ny + 1) * g.nz * g.nx;
  L.nh = (size_t)(g.ny + 1) * (g.nz + 1) * g.nx;
  L.n2 = (size_t)(g.ny + 1) * g.nx;
  L.state = v.state_bytes;
  const int nst = 3 * (v.msub + 1);
  size_t o = 0;
  L.traj_off = o; o += (size_t)nst * L.state;
  L.lam_off = o; o += 2 * L.state;
  L.f3_off = o; o += kN3 * a256(L.n3 * v.elem);
  L.fh_off = o; o += kNH * a256(L.nh * v.elem);
  L.f2t_off = o; o += kN2T * a256(L.n2 * v.elem);
  L.f2d_off = o; o += kN2D * a256(L.n2 * 8);
  L.psum_off = o; o += a256(8 * 2 * (g.nz + 1) * 8);
  L.pole_off = o; o += a256(4 * 2 * (g.nz + 1) * 8);
  L.tpole_off = o; o += a256((size_t)(nst + 1) * 2 * (g.nz + 1) * 8);   // pole values of each traj state
  L.total = o;
  return L;
}

template <typename T>
Scr<T> scratch_of(const HandleView& v, int set = 0) {
  const Layout L = layout(v);
  char* base = static_cast<char*>(v.adj);
  Scr<T> s;
  T* f3[kN3];
  for (int q = 0; q < kN3; ++q) f3[q] = reinterpret_cast<T*>(base + L.f3_off + q * a256(L.n3 * v.elem));
  s.RT = f3[0]; s.PHI = f3[1]; s.D = f3[2]; s.WP = f3[3];
  s.AVGL = f3[4]; s.AD = f3[5]; s.AFE = f3[6]; s.AP3 = f3[7]; s.HH = f3[8]; s.FU = f3[9];
  s.AUU = f3[10]; s.AUD = f3[11]; s.MV = f3[12]; s.FV = f3[13]; s.UV = f3[14]; s.AVV = f3[15]; s.AVD = f3[16];
  s.APU3 = f3[17]; s.APV3 = f3[18];
  s.APHI = f3[19]; s.ART = f3[20]; s.AL3 = f3[21]; s.AQ3 = f3[22]; s.ADL3 = f3[23]; s.ADQ3 = f3[24];
  s.UA = f3[25]; s.VT = f3[26];
  T* fh[kNH];
  for (int q = 0; q < kNH; ++q) fh[q] = reinterpret_cast<T*>(base + L.fh_off + q * a256(L.nh * v.elem));
  s.S = fh[0]; s.SD = fh[1]; s.ASD = fh[2];
  T* f2[kN2T];
  for (int q = 0; q < kN2T; ++q) f2[q] = reinterpret_cast<T*>(base + L.f2t_off + q * a256(L.n2 * v.elem));
  T** f2s = f2 + 5 * (set & 1);
  s.P = f2s[0]; s.L = f2s[1]; s.Q = f2s[2]; s.DL = f2s[3]; s.DQ = f2s[4];
  double* d2[kN2D];
  for (int q = 0; q < kN2D; ++q) d2[q] = reinterpret_cast<double*>(base + L.f2d_off + q * a256(L.n2 * 8));
  s.AP2 = d2[0]; s.APU2 = d2[1]; s.APV2 = d2[2]; s.AL2 = d2[3]; s.AQ2 = d2[4]; s.ADL2 = d2[5]; s.ADQ2 = d2[6];
  s.APSR = d2[7];
  s.psum = reinterpret_cast<double*>(base + L.psum_off);
  return s;
}

template <typename T>
struct St4 { T* U; T* V; T* F; T* P; };

template <typename T>
St4<T> state_at(const HandleView& v, void* base) {
  char* c = static_cast<char*>(base);
  St4<T> s;
  s.U = reinterpret_cast<T*>(c); c += a256(v.nU * sizeof(T));
  s.V = reinterpret_cast<T*>(c); c += a256(v.nV * sizeof(T));
  s.F = reinterpret_cast<T*>(c); c += a256(v.nF * sizeof(T));
  s.P = reinterpret_cast<T*>(c);
  return s;
}

// pin: pole values of y, formed here from y's pole rows unless pin_ready (the recorded forward's)
template <typename T>
// set: the set of 2D recompute fields the stage uses (f2d_ready: they hold its input's already);
// next_ps, next_pin: the next stage's input p_s and pole values, whose 2D recompute goes into the
// other set at the end of the pole-row chain when the stage forks one (*prefetched tells)
hipError_t stage_adjoint_impl(const HandleView& v, int process, double ch, St4<const T> y, St4<const T> ao,
                              St4<T> ab, St4<T> ai, double* pin, hipStream_t s, bool ai_zero = false,
                              bool pin_ready = false, int set = 0, bool f2d_ready = false,
                              const T* next_ps = nullptr, const double* next_pin = nullptr,
                              bool* prefetched = nullptr) {
  Ctx<T> c;
  c.g = v.g;
  c.U = y.U; c.V = y.V; c.F = y.F; c.P = y.P;
  c.aoU = ao.U; c.aoV = ao.V; c.aoF = ao.F; c.aoP = ao.P;
  c.abU = ab.U; c.abV = ab.V; c.abF = ab.F; c.abP = ab.P;
  c.aiU = ai.U; c.aiV = ai.V; c.aiF = ai.F; c.aiP = ai.P;
  c.pin = pin;
  c.ch = ch;
  c.s = scratch_of<T>(v, set);
  c.f = v.fac;
  c.blk = v.block;
  c.timer = v.timer;
  c.aat = v.aat;
  c.aat_n = v.aat_n;
  c.aat_blk = v.aat_block;
  c.aat_edge_n = v.aat_edge_n;
  c.side = v.adj_side;
  c.adt = v.adt;
  c.adt_n = v.adt_n;
  c.adt_blk = v.adt_block;
  c.pp_n = v.adt_pp_n;
  c.pp_s = v.adt_pp_s;
  c.ai_zero = ai_zero && ab.U != ai.U;
  c.base_in_tail = process == 1 && ab.U && ab.U == ai.U && ab.V == ai.V && ab.F == ai.F && ab.P == ai.P;
  c.f2d_ready = f2d_ready;
  const bool forks = process == 0 ? aar_split(c) && c.side != nullptr : adt_fork(c);
  if (forks && next_ps) {
    const Scr<T> o = scratch_of<T>(v, set + 1);
    c.next_ps = next_ps;
    c.next_pin = next_pin;
    c.next2d[0] = o.P; c.next2d[1] = o.L; c.next2d[2] = o.Q; c.next2d[3] = o.DL; c.next2d[4] = o.DQ;
  }
  if (prefetched) *prefetched = c.next_ps != nullptr;
  hipError_t e = pin_ready ? hipSuccess : launch_pole_prep<T>(v.g, y.F, y.P, pin, s);
  if (e != hipSuccess) return e;
  e = run_stage_adjoint<T>(c, s, process == 0);
  if (e != hipSuccess) return e;
  return process == 0 ? run_adapt<T>(c, s) : run_advect<T>(c, s);
}

template <typename T>
hipError_t zero_state(const HandleView& v, St4<T> a, hipStream_t s) {
  hipError_t e = launch_zero<T>(a.U, v.nU, s);
  if (e == hipSuccess) e = launch_zero<T>(a.V, v.nV, s);
  if (e == hipSuccess) e = launch_zero<T>(a.F, v.nF, s);
  if (e == hipSuccess) e = launch_zero<T>(a.P, v.nP, s);
  return e;
}

// Zeroes only what kernels other than the row-fused stage adjoints add to: the rows those leave to
// the per-point kernels (pole rows of U and Phi, V row 1/2, with the advection also rows 1..pp_n and
// ny-pp_s..ny-1 of U, V, Phi) and p_s.  The row-fused kernels store the other rows of an input
// adjoint the caller marks as zeroed (Ctx::ai_zero).
// The seven segments cleared in one launch: blockIdx.y picks the segment, the blocks along x stride
// over it (vector stores).
template <typename T>
struct ZeroSegs {
  T* p[7];
  unsigned n[7];
};

template <typename T>
__global__ void __launch_bounds__(256) k_zero_segs(ZeroSegs<T> z) {
  T* p = z.p[blockIdx.y];
  const unsigned n = z.n[blockIdx.y];
  for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) p[i] = T(0);
}

template <typename T>
hipError_t zero_outside_rows(const HandleView& v, St4<T> a, hipStream_t s, int pn, int ps) {
  const size_t row = (size_t)v.g.nz * v.g.nx, ny = (size_t)v.g.ny;
  const size_t nn = (size_t)(pn + 1) * row, ns = (size_t)(ps + 1) * row;   // rows 0..pn, ny-ps..ny
  const ZeroSegs<T> z{{a.U, a.U + (ny - ps) * row, a.F, a.F + (ny - ps) * row, a.V, a.V + (ny - ps) * row, a.P},
                      {(unsigned)nn, (unsigned)ns, (unsigned)nn, (unsigned)ns, (unsigned)nn,
                       (unsigned)(ns - row), (unsigned)v.nP}};
  const size_t most = std::max(std::max(nn, ns), v.nP);
  const unsigned gx = (unsigned)std::min<size_t>((most + 255) / 256, 1024);
  hipLaunchKernelGGL((k_zero_segs<T>), dim3(gx, 7), dim3(256), 0, s, z);
  return hipGetLastError();
}

// Whether a stage adjoint of this handle runs a row-fused kernel (as aar_used and adt_used): then the
// input adjoint's interior rows are stored without a read.
template <typename T>
bool rows_fused(const HandleView& v, int process) {
  Ctx<T> c;
  c.g = v.g;
  c.blk = v.block;
  c.aat = v.aat;
  c.aat_n = v.aat_n;
  c.adt = v.adt;
  c.adt_n = v.adt_n;
  return process == 0 ? aar_used(c) : adt_used(c);
}

template <typename T>
hipError_t copy_state(const HandleView& v, St4<T> d, St4<const T> src, hipStream_t s) {
  hipError_t e = launch_axpy_fill<T>(d.U, src.U, v.nU, s);
  if (e == hipSuccess) e = launch_axpy_fill<T>(d.V, src.V, v.nV, s);
  if (e == hipSuccess) e = launch_axpy_fill<T>(d.F, src.F, v.nF, s);
  if (e == hipSuccess) e = launch_axpy_fill<T>(d.P, src.P, v.nP, s);
  return e;
}

template <typename T>
St4<const T> cst(St4<T> a) { return St4<const T>{a.U, a.V, a.F, a.P}; }

// Forward pass of one outer step that keeps every stage input in the workspace: traj[3 rk] = y_rk,
// traj[3 rk + 1] = y1, traj[3 rk + 2] = y2, with their pole values (tpole[q]: those of y0 from its
// pole rows, the others as the stage that wrote the state formed them), which the reverse sweep
// linearises about.  With `out` set, the last stage of the last RK step is run too and writes the
// step's result there (out may be y0's buffers: y0 is copied first).
template <typename T>
int record_impl(const HandleView& v, St4<const T> y0, St4<T> out, hipStream_t s) {
  const Layout L = layout(v);
  char* base = static_cast<char*>(v.adj);
  const int nrk = v.msub + 1;
  auto traj = [&](int q) { return state_at<T>(v, base + L.traj_off + (size_t)q * L.state); };
  const size_t ps = 2 * (v.g.nz + 1);
  double* tp = reinterpret_cast<double*>(base + L.tpole_off);   // [3 nrk + 1][2][nz+1]
  auto tpole = [&](int q) { return tp + (size_t)q * ps; };
  hipError_t e;
  e = copy_state<T>(v, traj(0), y0, s);
  if (e != hipSuccess) return DYCORE_EHIP;
  e = launch_pole_prep<T>(v.g, traj(0).F, traj(0).P, tpole(0), s);
  if (e != hipSuccess) return DYCORE_EHIP;
  for (int rk = 0; rk < nrk; ++rk) {
    const int proc = rk < v.msub ? 0 : 1;
    const double h = proc == 0 ? v.dt / v.msub : v.dt;
    St4<T> y = traj(3 * rk), y1 = traj(3 * rk + 1), y2 = traj(3 * rk + 2);
    auto mk = [&](double chh, St4<T> in, St4<T> out, double* pin, double* pout) {
      StageArgs<T> a;
      a.g = v.g;
      a.inU = in.U; a.inV = in.V; a.inF = in.F; a.inP = in.P;
      a.bU = y.U; a.bV = y.V; a.bF = y.F; a.bP = y.P;
      a.oU = out.U; a.oV = out.V; a.oF = out.F; a.oP = out.P;
      a.pin = pin; a.pbase = tpole(3 * rk); a.pout = pout;
      a.ch = chh;
      a.process = proc;
      a.pad = 0;
      a.tiles = v.ftiles;
      a.cap = v.cap;
      a.ntiles = v.nftiles;
      a.tblock = v.ftblock;
      a.atiles = v.atiles;
      a.natiles = v.natiles;
      a.ablock = v.ablock;
      a.awide = v.awide;
      a.ptiles = v.ptiles;
      a.nptiles = v.nptiles;
      a.pblock = v.pblock;
      return a;
    };
    const int q = 3 * rk;
    e = launch_stage<T>(mk(h / 3.0, y, y1, tpole(q), tpole(q + 1)), s, v.side);
    if (e == hipSuccess) e = launch_stage<T>(mk(h / 2.0, y1, y2, tpole(q + 1), tpole(q + 2)), s, v.side);
    if (e == hipSuccess && rk + 1 < nrk) {
      e = launch_stage<T>(mk(h, y2, traj(q + 3), tpole(q + 2), tpole(q + 3)), s, v.side);
    } else if (e == hipSuccess && out.U) {
      // (the step result's pole values go to the spare last slot)
      e = launch_stage<T>(mk(h, y2, out, tpole(q + 2), tpole(q + 3)), s, v.side);
      // the low-latitude filters close the step, as in dycore_step
      if (e == hipSuccess) e = launch_lowlat<T>(v.g, v.filt, v.nfilt, out.U, out.V, out.F, out.P, s);
    }
    if (e != hipSuccess) return DYCORE_EHIP;
  }
  return DYCORE_OK;
}

// Reverse sweep over the stage inputs held in the workspace.
template <typename T>
int reverse_impl(const HandleView& v, St4<T> lam, hipStream_t s) {
  const Layout L = layout(v);
  char* base = static_cast<char*>(v.adj);
  const int nrk = v.msub + 1;
  auto traj = [&](int q) { return state_at<T>(v, base + L.traj_off + (size_t)q * L.state); };
  St4<T> l1 = state_at<T>(v, base + L.lam_off);
  St4<T> l2 = state_at<T>(v, base + L.lam_off + L.state);
  const size_t ps = 2 * (v.g.nz + 1);
  double* tp = reinterpret_cast<double*>(base + L.tpole_off);   // the recorded stage inputs' pole values
  auto tpole = [&](int q) { return tp + (size_t)q * ps; };
  // the low-latitude filters act last in the step and each row operator is symmetric, so the sweep
  // starts with the same filters applied to lam
  hipError_t e = launch_lowlat<T>(v.g, v.filt, v.nfilt, lam.U, lam.V, lam.F, lam.P, s);
  if (e != hipSuccess) return DYCORE_EHIP;
  // reverse sweep.  lam accumulates the adjoint of the RK step's input: every stage adds the base
  // transpose of its output adjoint to it; the last stage's share is lam itself with the base
  // transpose applied in place once that stage has read it.
  const St4<T> none{nullptr, nullptr, nullptr, nullptr};
  // the 2D recompute of each stage's input alternates between two sets; a stage that forks a pole-row
  // chain computes the next stage's at its end, and the next stage then skips it
  int set = 0;
  bool ready = false;
  for (int rk = nrk - 1; rk >= 0; --rk) {
    const int proc = rk < v.msub ? 0 : 1;
    const double h = proc == 0 ? v.dt / v.msub : v.dt;
    St4<T> y = traj(3 * rk), y1 = traj(3 * rk + 1), y2 = traj(3 * rk + 2);
    // l2 and l1 start at zero: where the row-fused kernel stores their interior rows, only the
    // rest is cleared
    const bool fused = rows_fused<T>(v, proc);
    const int pn = proc == 0 ? 0 : v.adt_pp_n, psn = proc == 0 ? 0 : v.adt_pp_s;
    e = fused ? zero_outside_rows<T>(v, l1, s, pn, psn) : zero_state<T>(v, l1, s);
    if (e == hipSuccess) e = fused ? zero_outside_rows<T>(v, l2, s, pn, psn) : zero_state<T>(v, l2, s);
    const int q = 3 * rk;
    // the input that the stage after the third one reads: the next RK step's third stage input
    const T* nps = rk > 0 ? traj(3 * (rk - 1) + 2).P : nullptr;
    const double* npin = rk > 0 ? tpole(3 * (rk - 1) + 2) : nullptr;
    bool pre = false;
    if (e == hipSuccess)
      e = stage_adjoint_impl<T>(v, proc, h, cst(y2), cst(lam), none, l2, tpole(q + 2), s, true, true, set, ready,
                                y1.P, tpole(q + 1), &pre);
    set ^= 1;
    ready = pre;
    if (e == hipSuccess) {
      hipLaunchKernelGGL((k_base_inplace<T>), dim3(v.g.nz + 1, 2), dim3(256), 0, s, v.g, lam.U, lam.F, lam.P);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = stage_adjoint_impl<T>(v, proc, h / 2.0, cst(y1), cst(l2), lam, l1, tpole(q + 1), s, true, true, set, ready,
                                y.P, tpole(q), &pre);
    set ^= 1;
    ready = pre;
    if (e == hipSuccess)
      e = stage_adjoint_impl<T>(v, proc, h / 3.0, cst(y), cst(l1), lam, lam, tpole(q), s, false, true, set, ready,
                                nps, npin, &pre);
    set ^= 1;
    ready = pre;
    if (e != hipSuccess) return DYCORE_EHIP;
  }
  return DYCORE_OK;
}

template <typename T>
int step_adjoint_impl(const HandleView& v, St4<const T> y0, St4<T> lam, hipStream_t s) {
  const St4<T> none{nullptr, nullptr, nullptr, nullptr};
  *v.recorded = 0;
  const int st = record_impl<T>(v, y0, none, s);
  return st != DYCORE_OK ? st : reverse_impl<T>(v, lam, s);
}

}  // namespace

size_t dyc_adjoint_workspace_bytes(const dycore_s* h) { return layout(view_of(h)).total; }

extern "C" {

int dycore_step_adjoint(dycore_t h, const void* U0, const void* V0, const void* Phi0, const void* ps0, void* aU,
                        void* aV, void* aPhi, void* aps, void* stream) {
  if (!h || !U0 || !V0 || !Phi0 || !ps0 || !aU || !aV || !aPhi || !aps) return DYCORE_EINVAL;
  const HandleView v = view_of(h);
  if (!v.adj) return DYCORE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (v.prec == DYCORE_FP32)
    return step_adjoint_impl<float>(v, St4<const float>{(const float*)U0, (const float*)V0, (const float*)Phi0,
                                                        (const float*)ps0},
                                    St4<float>{(float*)aU, (float*)aV, (float*)aPhi, (float*)aps}, s);
  return step_adjoint_impl<double>(v, St4<const double>{(const double*)U0, (const double*)V0, (const double*)Phi0,
                                                        (const double*)ps0},
                                   St4<double>{(double*)aU, (double*)aV, (double*)aPhi, (double*)aps}, s);
}

int dycore_step_record(dycore_t h, void* U, void* V, void* Phi, void* ps, void* stream) {
  if (!h || !U || !V || !Phi || !ps) return DYCORE_EINVAL;
  const HandleView v = view_of(h);
  if (!v.adj) return DYCORE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  *v.recorded = 0;
  int st;
  if (v.prec == DYCORE_FP32) {
    using T = float;
    st = record_impl<T>(v, St4<const T>{(const T*)U, (const T*)V, (const T*)Phi, (const T*)ps},
                        St4<T>{(T*)U, (T*)V, (T*)Phi, (T*)ps}, s);
  } else {
    using T = double;
    st = record_impl<T>(v, St4<const T>{(const T*)U, (const T*)V, (const T*)Phi, (const T*)ps},
                        St4<T>{(T*)U, (T*)V, (T*)Phi, (T*)ps}, s);
  }
  if (st == DYCORE_OK) *v.recorded = 1;
  return st;
}

int dycore_step_adjoint_recorded(dycore_t h, void* aU, void* aV, void* aPhi, void* aps, void* stream) {
  if (!h || !aU || !aV || !aPhi || !aps) return DYCORE_EINVAL;
  const HandleView v = view_of(h);
  if (!v.adj || !*v.recorded) return DYCORE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (v.prec == DYCORE_FP32)
    return reverse_impl<float>(v, St4<float>{(float*)aU, (float*)aV, (float*)aPhi, (float*)aps}, s);
  return reverse_impl<double>(v, St4<double>{(double*)aU, (double*)aV, (double*)aPhi, (double*)aps}, s);
}

int dycore_stage_adjoint(dycore_t h, int process, double ch, const void* U, const void* V, const void* Phi,
                         const void* ps, const void* aoU, const void* aoV, const void* aoPhi, const void* aops,
                         void* abU, void* abV, void* abPhi, void* abps, void* aiU, void* aiV, void* aiPhi,
                         void* aips, void* stream) {
  if (!h || (process != 0 && process != 1)) return DYCORE_EINVAL;
  const void* ptrs[16] = {U, V, Phi, ps, aoU, aoV, aoPhi, aops, abU, abV, abPhi, abps, aiU, aiV, aiPhi, aips};
  for (auto p : ptrs)
    if (!p) return DYCORE_EINVAL;
  const HandleView v = view_of(h);
  if (!v.adj) return DYCORE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout L = layout(v);
  double* pin = reinterpret_cast<double*>(static_cast<char*>(v.adj) + L.pole_off);
  hipError_t e;
  if (v.prec == DYCORE_FP32) {
    using T = float;
    e = stage_adjoint_impl<T>(v, process, ch, St4<const T>{(const T*)U, (const T*)V, (const T*)Phi, (const T*)ps},
                              St4<const T>{(const T*)aoU, (const T*)aoV, (const T*)aoPhi, (const T*)aops},
                              St4<T>{(T*)abU, (T*)abV, (T*)abPhi, (T*)abps}, St4<T>{(T*)aiU, (T*)aiV, (T*)aiPhi, (T*)aips},
                              pin, s);
  } else {
    using T = double;
    e = stage_adjoint_impl<T>(v, process, ch, St4<const T>{(const T*)U, (const T*)V, (const T*)Phi, (const T*)ps},
                              St4<const T>{(const T*)aoU, (const T*)aoV, (const T*)aoPhi, (const T*)aops},
                              St4<T>{(T*)abU, (T*)abV, (T*)abPhi, (T*)abps}, St4<T>{(T*)aiU, (T*)aiV, (T*)aiPhi, (T*)aips},
                              pin, s);
  }
  return e == hipSuccess ? DYCORE_OK : DYCORE_EHIP;
}

}  // extern "C"
