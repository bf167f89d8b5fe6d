// Forward stage kernels of the leap-format dynamical core (gfx950).
//
// One workgroup owns one latitude row j: the scalar row j (Phi, p_s), the U
// row j and the V row j+1/2.  It walks the column top to bottom, level by
// level; each thread owns columns i = t, t+B, ... of the row and keeps its
// column sums in FP64 registers.  Rows that a leap difference reads at
// distance up to M (eq. 6, Table VII) are staged whole in LDS, so the periodic
// zonal wrap is a modular index into LDS and never a halo exchange.  Pole rows
// are reduced in FP64 by the first wavefront in a fixed lane order, so results
// do not depend on the workgroup size.
#include "dycore_internal.h"

namespace dyc {
namespace {

template <typename T> __device__ __forceinline__ T tsqrt(T x);
template <> __device__ __forceinline__ float tsqrt<float>(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double tsqrt<double>(double x) { return sqrt(x); }
template <typename T> __device__ __forceinline__ T tlog(T x);
template <> __device__ __forceinline__ float tlog<float>(float x) { return logf(x); }
template <> __device__ __forceinline__ double tlog<double>(double x) { return log(x); }

__device__ __forceinline__ int wrp(int i, int nx) {
  // |offset| < nx for every caller
  return i >= nx ? i - nx : (i < 0 ? i + nx : i);
}
// one-sided forms, where the offset's sign is known: 0 <= i < 2 nx, and -nx <= i < nx
__device__ __forceinline__ int wrp_up(int i, int nx) { return i >= nx ? i - nx : i; }
__device__ __forceinline__ int wrp_dn(int i, int nx) { return i < 0 ? i + nx : i; }

// Deterministic FP64 row sum by wavefront 0: lane l adds i = l, l+64, ... in
// order, then a butterfly (commutative adds give every lane the same total).
__device__ __forceinline__ double wave_sum(double acc) {
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  return acc;
}

using C = double;

// A global load or store at the array's base plus a 32-bit element offset (fields hold fewer than
// 2^30 elements; create refuses larger grids).
template <typename T>
__device__ __forceinline__ T ldg(const T* p, unsigned idx) {
  return *(const __attribute__((address_space(1))) T*)(
      (const __attribute__((address_space(1))) char*)p + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stg(T* p, unsigned idx, T v) {
  *(__attribute__((address_space(1))) T*)((__attribute__((address_space(1))) char*)p + idx * (unsigned)sizeof(T)) = v;
}

}  // namespace

// kappa* D_sa of eq. 1's p_s line at column i of interior row j, from the stage input's stored p_s
// (pole values read from their slot), FP64: the flux-form horizontal Laplacian, zonally the leaped
// second difference (F_{i+M} - 2 F_i + F_{i-M}) / (M dx)^2, meridionally the difference of the face
// gradients times sin(theta) at the faces over a^2 sin(theta_j) dtheta^2.
template <typename T>
__device__ __forceinline__ C ps_diffusion(const StageArgs<T>& A, int j, int i) {
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  auto ps = [&](int jr, int ii) -> C {
    if (jr == 0) return A.pin[nz];
    if (jr == ny) return A.pin[(nz + 1) + nz];
    return (C)A.inP[(size_t)jr * nx + ii];
  };
  const int M = g.M[j];
  const C dx = (C)M * g.a * g.s[j] * g.dlam;
  const C dy2 = g.a * g.a * g.s[j] * g.dth * g.dth;
  const C p0 = ps(j, i);
  const C zon = (ps(j, wrp(i + M, nx)) - 2.0 * p0 + ps(j, wrp(i - M, nx))) / (dx * dx);
  const C mer = (g.sv[j] * (ps(j + 1, i) - p0) - g.sv[j - 1] * (p0 - ps(j - 1, i))) / dy2;
  return g.kstar * (zon + mer);
}

// kappa* D_sa at a pole: the outward gradient flux through the cap edge over the cap area,
// sin(theta_1/2) dlam / (A_cap dtheta) sum_i (p_s(adjacent row, i) - p_pole), summed in FP64 in a
// fixed order by wavefront 0 and returned to every thread (a workgroup-wide barrier inside).
template <typename T>
__device__ C ps_diffusion_pole(const StageArgs<T>& A, int j, double* red) {
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ja = (j == 0) ? 1 : ny - 1, jv = (j == 0) ? 0 : ny - 1;
  const C pp = A.pin[(j == 0 ? 0 : nz + 1) + nz];
  if (threadIdx.x < 64) {
    C s = 0;
    for (int i = threadIdx.x; i < nx; i += 64) s += (C)A.inP[(size_t)ja * nx + i] - pp;
    s = wave_sum(s);
    if (threadIdx.x == 0) red[0] = s;
  }
  __syncthreads();
  return g.kstar * (g.sv[jv] * g.dlam / (g.acap * g.dth)) * red[0];
}


namespace {

// ----------------------------------------------------------------------------------------------
// Adaptation: out = base + ch * A(in)
// ----------------------------------------------------------------------------------------------
// Per zonal slot, the LDS holds 13 2D rows (P, the reciprocals of P and of its U-point averages,
// the leaped d+l and d+q, the V-point averages of P, the meridional l and q differences) and,
// double-buffered, the 7 per-level rows (phi', MU, Phi, U of rows j and j+1, V of rows j+-1/2).
constexpr int kAdaptPipeRows2D = 13, kAdaptPipeRowsLev = 7;

// Adaptation, tiled: one workgroup per work item (row j, a zonal tile of w owned columns from i0 and
// a halo of hl = n_j + 1 columns on each side), one column per thread.  The stage's arithmetic is
// that of the pipelined row form: every value a level reads at another column sits in LDS, per slot
// 27 words (the 13 2D rows, then two buffers of the 7 level rows; an odd stride, no bank conflicts),
// level k+1 is fetched into registers while level k is computed, one barrier per level.  The leap
// and +-1 neighbours of the owned columns are halo slots, so LDS indices need no wrap, and a tile's
// small LDS leaves room for several workgroups per CU.  Pole rows (j = 0, ny) take their cap sums from
// k_capsum, which runs before the stage; their tiles write the replicated pole values of their own
// columns.
constexpr int kTileRS = kAdaptPipeRows2D + 2 * kAdaptPipeRowsLev;   // 27 words per slot
__host__ __device__ constexpr size_t adapt_tile_lds(int block, int elem) {
  return (size_t)kTileRS * block * elem + 8 * sizeof(double);
}

template <typename T>
__device__ void adapt_tile(const StageArgs<T>& A, const AatItem it, unsigned char* smem) {
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int j = it.j, hl = it.hl, w = it.w;
  const int NS = w + 2 * hl;
  const int sl = threadIdx.x;
  const bool act = sl < NS;
  const bool own = sl >= hl && sl < hl + w;
  int col = (it.i0 - hl + sl) % nx;
  if (col < 0) col += nx;
  const int colp = col == nx - 1 ? 0 : col + 1;
  T* r = reinterpret_cast<T*>(smem);
  double* red = reinterpret_cast<double*>(smem + (size_t)kTileRS * blockDim.x * sizeof(T));
  auto S2 = [&](int row, int slot) -> T& { return r[slot * kTileRS + row]; };
  auto SB = [&](int bsel, int row, int slot) -> T& {
    return r[slot * kTileRS + kAdaptPipeRows2D + bsel * kAdaptPipeRowsLev + row];
  };
  enum { RP0, RrP0, RrP1, RrU0, RrU1, RDl, RDq, RPV0, RPVm, RgN, RgS, RdL, RdQ };
  enum { BPhi, BMU, BF, BU0, BU1, BV0, BVm };

  const bool isPole = (j == 0 || j == ny);
  const bool hasV = (j < ny);
  const int pidx = (j == 0) ? 0 : 1;
  const T p0 = (T)g.p0, b = (T)g.b, RT0 = (T)g.RT0;
  const C RT0c = g.RT0;
  const unsigned row3 = (unsigned)(nz * nx);
  auto psA = [&](int jr, int i) -> T {
    if (jr == 0) return (T)A.pin[nz];
    if (jr == ny) return (T)A.pin[(nz + 1) + nz];
    return A.inP[(size_t)jr * nx + i];
  };

  // ---- 2D rows of every slot (l and q of row j in buffer 0 until the leaped differences are formed)
  if (act) {
    const T ps0 = psA(j, col);
    const T P0 = tsqrt<T>(ps0 / p0), L0 = tlog<T>(ps0 / p0);
    const T Q0 = L0 + (T)g.phis[(size_t)j * nx + col] / RT0;
    const T P0p = tsqrt<T>(psA(j, colp) / p0);
    S2(RP0, sl) = P0;
    S2(RrP0, sl) = T(1) / P0;
    S2(RrU0, sl) = T(2) / (P0 + P0p);
    SB(0, 1, sl) = L0;
    SB(0, 2, sl) = Q0;
    if (hasV) {
      const T ps1 = psA(j + 1, col);
      const T P1 = tsqrt<T>(ps1 / p0), L1 = tlog<T>(ps1 / p0);
      const T Q1 = L1 + (T)g.phis[(size_t)(j + 1) * nx + col] / RT0;
      const T P1p = tsqrt<T>(psA(j + 1, colp) / p0);
      S2(RrP1, sl) = T(1) / P1;
      S2(RrU1, sl) = T(2) / (P1 + P1p);
      const T PV0 = T(0.5) * (P0 + P1);
      S2(RPV0, sl) = PV0;
      S2(RgN, sl) = (L1 - L0) / PV0;
      S2(RdL, sl) = L1 - L0;
      S2(RdQ, sl) = Q1 - Q0;
    }
    if (j >= 1) {
      const T psm = psA(j - 1, col);
      const T Pm = tsqrt<T>(psm / p0), Lm = tlog<T>(psm / p0);
      const T PVm = T(0.5) * (Pm + P0);
      S2(RPVm, sl) = PVm;
      S2(RgS, sl) = (L0 - Lm) / PVm;
    }
  }
  __syncthreads();
  const int Mj = isPole ? 1 : g.M[j];
  const int nj = (Mj + 1) / 2;
  const T rdx = isPole ? T(0) : (T)(1.0 / ((double)Mj * g.a * g.s[j] * g.dlam));
  if (!isPole && sl >= nj - 1 && sl + nj < NS) {   // the slots whose leap neighbours are in the tile
    S2(RDl, sl) = (SB(0, 1, sl + nj) - SB(0, 1, sl + 1 - nj)) * rdx;
    S2(RDq, sl) = (SB(0, 2, sl + nj) - SB(0, 2, sl + 1 - nj)) * rdx;
  }
  __syncthreads();

  // ---- pass A: column totals of R T' (the hydrostatic suffix sums start from them)
  C Q0c = 0, Q1c = 0, Sc = 0;
  if (hasV && act) {
    const T rp0 = b * S2(RrP0, sl), rp1 = b * S2(RrP1, sl);
    constexpr int KU = 6;
    for (int k0 = 0; k0 < nz; k0 += KU) {
      T f0[KU], f1[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + u < nz ? k0 + u : nz - 1;
        const unsigned o = (unsigned)(k * nx + col);
        f0[u] = isPole ? (T)A.pin[k] : ldg(A.inF, (unsigned)j * row3 + o);
        f1[u] = (j + 1 < ny) ? ldg(A.inF, (unsigned)(j + 1) * row3 + o) : (T)A.pin[(nz + 1) + k];
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        if (k0 + u >= nz) break;
        const C clk = g.cl[k0 + u];
        Q0c += clk * (C)(f0[u] * rp0);
        Q1c += clk * (C)(f1[u] * rp1);
      }
    }
  }

  // ---- pass B, pipelined over levels: the next level's inputs and base values are fetched while
  // the current level is computed
  T nF0 = 0, nF1 = 0, nU0 = 0, nU1 = 0, nV0 = 0, nVm = 0;
  T nbF = 0, nbU = 0, nbV = 0;
  auto fetch = [&](int k) {
    if (!act) return;
    const unsigned lo = (unsigned)j * row3 + (unsigned)(k * nx + col);
    if (own) {
      if (!isPole) {
        nbF = ldg(A.bF, lo);
        nbU = ldg(A.bU, lo);
      }
      if (hasV) nbV = ldg(A.bV, lo);
    }
    nF0 = isPole ? (T)A.pin[pidx * (nz + 1) + k] : ldg(A.inF, lo);
    nU0 = isPole ? T(0) : ldg(A.inU, lo);
    nF1 = (j + 1 < ny) ? ldg(A.inF, lo + row3) : (T)A.pin[(nz + 1) + k];
    nU1 = (j + 1 < ny) ? ldg(A.inU, lo + row3) : T(0);
    nV0 = hasV ? ldg(A.inV, lo) : T(0);
    nVm = (j >= 1) ? ldg(A.inV, lo - row3) : T(0);
  };
  // R T' and phi' of rows j and j+1 at the current level (registers)
  T RTj = 0, RTj1 = 0, phij = 0, phij1 = 0;
  auto commit = [&](int k, int bs) {
    if (!act) return;
    const C clk = g.cl[k], cpk = g.cpk[k];
    RTj = b * nF0 * S2(RrP0, sl);
    SB(bs, BF, sl) = nF0;
    SB(bs, BU0, sl) = nU0;
    // (the last slot's MU is never gathered; its eastern neighbour is out of the tile)
    SB(bs, BMU, sl) = T(0.5) * (S2(RP0, sl) + S2(RP0, sl + 1 < NS ? sl + 1 : sl)) * nU0;
    RTj1 = phij = phij1 = T(0);
    if (hasV) {
      Q0c -= clk * (C)RTj;
      phij = (T)(Q0c + cpk * (C)RTj);
      RTj1 = b * nF1 * S2(RrP1, sl);
      Q1c -= clk * (C)RTj1;
      phij1 = (T)(Q1c + cpk * (C)RTj1);
      SB(bs, BU1, sl) = nU1;
      SB(bs, BV0, sl) = nV0;
    }
    SB(bs, BVm, sl) = nVm;
    SB(bs, BPhi, sl) = phij;
  };

  fetch(0);
  commit(0, 0);
  __syncthreads();

  C Sp = 0;
  const T rdyS = isPole ? T(0) : (T)(1.0 / (g.a * g.s[j] * g.dth));
  const T rdyA = (T)(1.0 / (g.a * g.dth));
  const C rdyAc = 1.0 / (C)(T)(g.a * g.dth);
  const T svj = isPole ? T(0) : (T)g.sv[j], svm = isPole ? T(0) : (T)g.sv[j - 1];
  const T fj = (T)g.f[j], cota = (T)(g.cot[j] / g.a);
  const T kap = (T)g.kappa;
  const T fvj = hasV ? (T)g.fv[j] : T(0), cotva = hasV ? (T)(g.cotv[j] / g.a) : T(0);
  const double* cap = A.cap + pidx * 2 * nz;
  const unsigned oc = (unsigned)col;
#pragma unroll 1
  for (int k = 0; k < nz; ++k) {
    const T baseF = nbF, baseU = nbU, baseV = nbV;
    if (k + 1 < nz) fetch(k + 1);
    const int bs = k & 1;
    const C dsg = g.dsig[k], rsg = 1.0 / g.sig[k];
    const unsigned lo = (unsigned)j * row3 + (unsigned)(k * nx);
    if (own) {
      const int sp = sl + 1, sm = sl - 1;
      if (!isPole) {
        const T Vn = SB(bs, BV0, sl), Vs = SB(bs, BVm, sl);
        const T D = (SB(bs, BMU, sl + nj - 1) - SB(bs, BMU, sl - nj)) * rdx +
                    (svj * (S2(RPV0, sl) * Vn) - svm * (S2(RPVm, sl) * Vs)) * rdyS;
        const C Sk = Sc;
        Sc += (C)D * dsg;
        const T u_i = SB(bs, BU0, sl) * S2(RrU0, sl);
        const T u_m = SB(bs, BU0, sm) * S2(RrU0, sm);
        const T zon = T(0.5) * (u_i * S2(RDl, sl) + u_m * S2(RDl, sm));
        const T mer = T(0.5) * (Vn * S2(RgN, sl) + Vs * S2(RgS, sl)) * rdyA;
        const C rp = (C)S2(RrP0, sl);
        const C wp = ((C)zon + (C)mer) - (Sk + 0.5 * (C)D * dsg) * rsg * (rp * rp);
        const C TF = ((C)(b * S2(RP0, sl)) + (C)(kap * SB(bs, BF, sl))) * wp;
        stg(A.oF, lo + oc, (T)((C)baseF + A.ch * TF));
        const T dphi = (SB(bs, BPhi, sl + nj) - SB(bs, BPhi, sl + 1 - nj)) * rdx;
        const T rtx = T(0.5) * (RTj + b * SB(bs, BF, sp) * S2(RrP0, sp));
        const C pgf = (C)dphi + RT0c * (C)S2(RDq, sl) + (C)rtx * (C)S2(RDl, sl);
        const T VV = T(0.25) * (Vn + SB(bs, BV0, sp) + Vs + SB(bs, BVm, sp));
        const T fs = fj + u_i * cota;
        const C TU = -(C)(T(0.5) * (S2(RP0, sl) + S2(RP0, sp))) * pgf - (C)fs * (C)VV;
        stg(A.oU, lo + oc, (T)((C)baseU + A.ch * TU));
      } else {
        const T F0p = (T)A.pin[pidx * (nz + 1) + k];
        const int jva = (j == 0) ? 0 : ny - 1;
        const T Pp = S2(RP0, sl);
        const C sgn = (j == 0) ? 1.0 : -1.0;
        const C Dp = sgn * g.a * g.dlam * g.sv[jva] * cap[k] / g.acap;
        const C vglp = cap[nz + k] / ((double)nx * g.a * g.dth);
        const C Sk = Sp;
        Sp += Dp * dsg;
        const C wp = vglp - (Sk + 0.5 * Dp * dsg) * rsg / ((C)Pp * (C)Pp);
        const C TF = ((C)(b * Pp) + (C)(kap * F0p)) * wp;
        const T val = (T)(A.pbase[pidx * (nz + 1) + k] + A.ch * TF);
        stg(A.oF, lo + oc, val);
        stg(A.oU, lo + oc, T(0));
        if (col == 0) A.pout[pidx * (nz + 1) + k] = (double)val;
      }
      if (hasV) {
        const C pgf = ((C)(phij1 - phij) + RT0c * (C)S2(RdQ, sl) +
                       (C)(T(0.5) * (RTj + RTj1)) * (C)S2(RdL, sl)) * rdyAc;
        const T U0i = SB(bs, BU0, sl), U0m = SB(bs, BU0, sm), U1i = SB(bs, BU1, sl), U1m = SB(bs, BU1, sm);
        const T u0i = U0i * S2(RrU0, sl), u0m = U0m * S2(RrU0, sm);
        const T u1i = U1i * S2(RrU1, sl), u1m = U1m * S2(RrU1, sm);
        const T UU = T(0.25) * (U0m + U0i + U1m + U1i);
        const T uu = T(0.25) * (u0m + u0i + u1m + u1i);
        const T fs = fvj + uu * cotva;
        const C TV = -(C)S2(RPV0, sl) * pgf + (C)fs * (C)UU;
        stg(A.oV, lo + oc, (T)((C)baseV + A.ch * TV));
      }
    }
    if (k + 1 < nz) commit(k + 1, (k + 1) & 1);
    __syncthreads();
  }

  // surface pressure: -p0 * Pi (plus kappa* D_sa)
  if (!isPole) {
    if (own) {
      const size_t idx = (size_t)j * nx + col;
      const C dsa = g.kstar != 0.0 ? ps_diffusion(A, j, col) : 0.0;
      A.oP[idx] = (T)((C)A.bP[idx] + A.ch * (-g.p0 * Sc + dsa));
    }
  } else {
    const C dsa = g.kstar != 0.0 ? ps_diffusion_pole(A, j, red) : 0.0;
    const T val = (T)(A.pbase[pidx * (nz + 1) + nz] + A.ch * (-g.p0 * Sp + dsa));
    if (own) {
      A.oP[(size_t)j * nx + col] = val;
      if (col == 0) A.pout[pidx * (nz + 1) + nz] = (double)val;
    }
  }
}

// FP64 cap sums of the adaptation stage's input, one block per (level, pole): the flux
// sum_i P^V V through the V row next to the pole and sum_i (V / P^V) (l_adj - l_pole), in a fixed
// order (thread-strided partial sums, a butterfly per wavefront, the wavefronts in order), for the
// pole rows of adapt_tile.
constexpr int kCapChunk = 8;   // columns per thread whose loads go out together
constexpr int kCapBlock = 256;  // threads of a cap-sum block

// The block's two cap sums of one (level, pole): each wavefront's butterfly, then the wavefronts'
// sums added in wavefront order.
template <typename T>
__device__ __forceinline__ void cap_store(const StageArgs<T>& A, int k, int p, double s1, double s2) {
  __shared__ double red[2][kCapBlock / 64];
  const int nz = A.g.nz;
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s1;
    red[1][threadIdx.x >> 6] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t1 = 0, t2 = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      t1 += red[0][w];
      t2 += red[1][w];
    }
    A.cap[p * 2 * nz + k] = t1;
    A.cap[p * 2 * nz + nz + k] = t2;
  }
}

template <typename T>
__device__ void capsum_level(const StageArgs<T>& A, int k, int p) {
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const T p0 = (T)g.p0;
  const int ja = (p == 0) ? 1 : ny - 1, jva = (p == 0) ? 0 : ny - 1;
  const T pps = (T)A.pin[(p == 0 ? 0 : nz + 1) + nz];
  const T Pp = tsqrt<T>(pps / p0), lp = tlog<T>(pps / p0);
  const T* pV = A.inV + ((size_t)jva * nz + k) * nx;
  const T* pP = A.inP + (size_t)ja * nx;
  C s1 = 0, s2 = 0;
  // the thread's columns in index order, the loads of kCapChunk of them ahead of their additions
  const int nt = blockDim.x;
  for (int i0 = threadIdx.x; i0 < nx; i0 += nt * kCapChunk) {
    T psv[kCapChunk], vvv[kCapChunk];
#pragma unroll
    for (int u = 0; u < kCapChunk; ++u) {
      const int i = i0 + nt * u < nx ? i0 + nt * u : i0;
      psv[u] = pP[i];
      vvv[u] = pV[i];
    }
#pragma unroll
    for (int u = 0; u < kCapChunk; ++u) {
      if (i0 + nt * u >= nx) break;
      const T psa = psv[u];
      const T Pa = tsqrt<T>(psa / p0), La = tlog<T>(psa / p0);
      const T pv = T(0.5) * (Pp + Pa);
      const T vv = vvv[u];
      s1 += (C)(pv * vv);
      s2 += (C)((vv / pv) * (p == 0 ? (La - lp) : (lp - La)));
    }
  }
  cap_store(A, k, p, s1, s2);
}

template <typename T>
__global__ void __launch_bounds__(kCapBlock) k_capsum(StageArgs<T> a) {
  capsum_level<T>(a, blockIdx.x, blockIdx.y);
}


// ----------------------------------------------------------------------------------------------
// Advection, tiled: one workgroup per work item (row j, a zonal tile of w owned columns from i0,
// one column per thread).  Band tiles carry a halo of hl = max(M_j, Mv_j, 1) columns on each side,
// the reach of the leaped centred differences (2 M wide), and gather every level value from LDS.
// Wide tiles (rows whose halo would leave fewer than 32 owned columns in 256 threads: next to the
// poles on fine grids; marked hl < 0) keep a halo of one column and read their leap operands from
// global memory, forming u = U / P^U and the V-row mean of u there as the LDS rows hold them, so both
// forms give the same values.  Per slot the LDS holds, double-buffered, 7 level rows (Phi, U, u of
// row j, V, u on the V row, v sin(theta) on V rows j+-1/2) and a 3-slot sigma-dot ring: 17 words, an
// odd stride.  sigma-dot of row j comes from every slot's column total Pi (pass A, the leap
// neighbours of U from global memory) and running S; that of row j+1 is formed at the owned columns
// only.  The pole rows' cap sums come from k_capsum_adv.
// ----------------------------------------------------------------------------------------------
constexpr int kAdvTileRows = 7;
constexpr int kAdvTileRS = 2 * kAdvTileRows + 3;   // 17 words per slot
__host__ __device__ constexpr size_t advect_tile_lds(int block, int elem) { return (size_t)kAdvTileRS * block * elem; }

// WPF (wide tiles only): the leap operands and base values of level k+1 are fetched while level k is
// computed; without it a wide tile loads them at their level (the batched kernel's register budget)
template <typename T, bool WIDE, bool WPF = WIDE>
__device__ void advect_tile(const StageArgs<T>& A, const AatItem it, unsigned char* smem) {
  static_assert(WIDE || !WPF, "the prefetch serves wide tiles");
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int j = it.j, w = it.w, hl = WIDE ? 1 : it.hl;
  const int NS = w + 2 * hl;
  const int sl = threadIdx.x;
  const bool act = sl < NS;                  // slots past NS only meet the barriers
  const bool own = sl >= hl && sl < hl + w;  // owned column: the tendencies and every global write
  int col = (it.i0 - hl + sl) % nx;
  if (col < 0) col += nx;
  T* r = reinterpret_cast<T*>(smem);
  auto SB = [&](int bsel, int row, int slot) -> T& { return r[slot * kAdvTileRS + bsel * kAdvTileRows + row]; };
  auto SD = [&](int ring, int slot) -> T& { return r[slot * kAdvTileRS + 2 * kAdvTileRows + ring]; };
  enum { BF, BU, Bu0, BV, Buv, Bvt0, Bvtm };

  const bool isPole = (j == 0 || j == ny);
  const bool hasV = (j < ny);
  const bool j1Pole = (j + 1 == ny);
  const bool j1Int = (j + 1 >= 1 && j + 1 <= ny - 1);
  const int pidx = (j == 0) ? 0 : 1;
  const int ja = (j == 0) ? 1 : ny - 1;
  const T p0 = (T)g.p0;
  const unsigned row3 = (unsigned)(nz * nx);
  auto psA = [&](int jr, int i) -> T {
    if (jr == 0) return (T)A.pin[nz];
    if (jr == ny) return (T)A.pin[(nz + 1) + nz];
    return A.inP[(size_t)jr * nx + i];
  };
  auto Prow = [&](int jr, int i) -> T { return tsqrt<T>(psA(jr, i) / p0); };
  auto up1 = [&](int i) { return i == nx - 1 ? 0 : i + 1; };

  const int Mj = isPole ? 1 : g.M[j], nj = (Mj + 1) / 2;
  const int Mj1 = j1Int ? g.M[j + 1] : 1, nj1 = (Mj1 + 1) / 2;
  const T rdx = isPole ? T(0) : (T)(1.0 / ((double)Mj * g.a * g.s[j] * g.dlam));
  const T rdx1 = j1Int ? (T)(1.0 / ((double)Mj1 * g.a * g.s[j + 1] * g.dlam)) : T(0);
  const T rdyS = isPole ? T(0) : (T)(1.0 / (g.a * g.s[j] * g.dth));
  const T rdyS1 = j1Int ? (T)(1.0 / (g.a * g.s[j + 1] * g.dth)) : T(0);
  const T svj = hasV ? (T)g.sv[j] : T(0), svm = (j >= 1) ? (T)g.sv[j - 1] : T(0);
  const T sv1 = (j + 1 < ny) ? (T)g.sv[j + 1] : T(0);
  const C capD0 = isPole ? ((j == 0) ? 1.0 : -1.0) * g.a * g.dlam * g.sv[(j == 0) ? 0 : ny - 1] / g.acap : 0.0;
  const C capD1 = (hasV && j1Pole) ? -g.a * g.dlam * g.sv[ny - 1] / g.acap : 0.0;
  const double* cap0 = A.cap + pidx * 2 * nz;   // this pole row's sums (pole rows)
  const double* cap1 = A.cap + 1 * 2 * nz;      // the south pole's (row ny-1)

  // sigma-dot of row j: the owned columns and their eastern neighbour (the U points read both)
  const bool sdr = act && sl >= hl && sl <= hl + w;
  // ---- 2D values of this slot's column: P of rows j and j+1 (here and east), the U-point and
  // V-point factors, the P averages at the leap neighbours that the divergence reads
  const int ic = (col + nj - 1) % nx, id = (col - nj + nx) % nx;
  const int ic1 = (col + nj1 - 1) % nx, id1 = (col - nj1 + nx) % nx;
  T rPU0 = 0, rPU1 = 0, PV0 = 1, PVm = 1, PV1 = 1, rPV0 = 1, rPVm = 1, rPV1 = 1;
  T PUc = 0, PUd = 0, PU1c = 0, PU1d = 0;
  C rP0sq = 0, rP1sq = 0;
  if (act) {
    const T P0 = Prow(j, col), P1 = Prow(hasV ? j + 1 : ja, col);
    if (!isPole) rPU0 = T(2) / (P0 + Prow(j, up1(col)));
    if (j1Int) rPU1 = T(2) / (P1 + Prow(j + 1, up1(col)));
    if (hasV) PV0 = T(0.5) * (P0 + P1);
    if (j >= 1) PVm = T(0.5) * (Prow(j - 1, col) + P0);
    if (j + 2 <= ny) PV1 = T(0.5) * (P1 + Prow(j + 2, col));
    rPV0 = T(1) / PV0;
    rPVm = T(1) / PVm;
    rPV1 = T(1) / PV1;
    rP0sq = 1.0 / ((C)P0 * (C)P0);
    rP1sq = hasV ? 1.0 / ((C)P1 * (C)P1) : 0.0;
    if (sdr && !isPole) {
      PUc = T(0.5) * (Prow(j, ic) + Prow(j, up1(ic)));
      PUd = T(0.5) * (Prow(j, id) + Prow(j, up1(id)));
    }
    if (j1Int && own) {
      PU1c = T(0.5) * (Prow(j + 1, ic1) + Prow(j + 1, up1(ic1)));
      PU1d = T(0.5) * (Prow(j + 1, id1) + Prow(j + 1, up1(id1)));
    }
  }
  const bool d1 = own && hasV;   // sigma-dot of row j+1: owned columns only
  // divergence of rows j and j+1 at level k
  auto div0 = [&](int k, T Uic, T Uid, T Vj, T Vm) -> C {
    if (isPole) return capD0 * cap0[k];
    return (C)((PUc * Uic - PUd * Uid) * rdx + (svj * (PV0 * Vj) - svm * (PVm * Vm)) * rdyS);
  };
  auto div1 = [&](int k, T U1ic, T U1id, T Vj, T V1) -> C {
    if (!hasV) return 0.0;
    if (j1Pole) return capD1 * cap1[k];
    return (C)((PU1c * U1ic - PU1d * U1id) * rdx1 + (sv1 * (PV1 * V1) - svj * (PV0 * Vj)) * rdyS1);
  };
  auto gU = [&](int jr, int k, int i) -> T { return ldg(A.inU, (unsigned)jr * row3 + (unsigned)(k * nx + i)); };
  auto gV = [&](int jr, int k, int i) -> T { return ldg(A.inV, (unsigned)jr * row3 + (unsigned)(k * nx + i)); };
  auto gF = [&](int jr, int k, int i) -> T { return ldg(A.inF, (unsigned)jr * row3 + (unsigned)(k * nx + i)); };

  // ---- pass A: column totals Pi of rows j and j+1
  C Pi0 = 0, Pi1 = 0;
  if (sdr) {
    constexpr int KU = 3;
    for (int k0 = 0; k0 < nz; k0 += KU) {
      T a0[KU], a1[KU], a2[KU], a3[KU], a4[KU], a5[KU], a6[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + u < nz ? k0 + u : nz - 1;
        a0[u] = isPole ? T(0) : gU(j, k, ic);
        a1[u] = isPole ? T(0) : gU(j, k, id);
        a2[u] = (d1 && j1Int) ? gU(j + 1, k, ic1) : T(0);
        a3[u] = (d1 && j1Int) ? gU(j + 1, k, id1) : T(0);
        a4[u] = hasV ? gV(j, k, col) : T(0);
        a5[u] = (j >= 1) ? gV(j - 1, k, col) : T(0);
        a6[u] = (d1 && j + 1 < ny) ? gV(j + 1, k, col) : T(0);
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + u;
        if (k < nz) {
          const C dsg = g.dsig[k];
          Pi0 += div0(k, a0[u], a1[u], a4[u], a5[u]) * dsg;
          if (d1) Pi1 += div1(k, a2[u], a3[u], a4[u], a6[u]) * dsg;
        }
      }
    }
  }

  // ---- pass B, pipelined over levels: level k+1 is fetched while level k is computed
  T nF = 0, nU = 0, nV = 0, nVm = 0, nU1 = 0, nV1 = 0, nFn = 0, nFs = 0, nUs = 0;
  T nUic = 0, nUid = 0, nU1ic = 0, nU1id = 0;
  T cVm = 0, cU1 = 0, cV1 = 0, cFn = 0, cFs = 0, cUs = 0;   // the owned column's values at level k
  C S0 = 0, S1 = 0, sd0c = 0, sd0n = 0, sd1c = 0, sd1n = 0;
  auto fetch = [&](int k) {
    if (!act) return;
    nF = isPole ? (T)A.pin[pidx * (nz + 1) + k] : gF(j, k, col);
    nU = isPole ? T(0) : gU(j, k, col);
    nV = hasV ? gV(j, k, col) : T(0);
    nVm = (j >= 1) ? gV(j - 1, k, col) : T(0);
    nU1 = j1Int ? gU(j + 1, k, col) : T(0);
    if (sdr && !isPole) {
      nUic = gU(j, k, ic);
      nUid = gU(j, k, id);
    }
    if (own) {
      nV1 = (j + 1 < ny) ? gV(j + 1, k, col) : T(0);
      nFn = (!isPole && j + 1 < ny) ? gF(j + 1, k, col) : ((j + 1 == ny) ? (T)A.pin[(nz + 1) + k] : T(0));
      nFs = (!isPole && j - 1 >= 1) ? gF(j - 1, k, col) : ((j - 1 == 0) ? (T)A.pin[k] : T(0));
      nUs = (!isPole && j - 1 >= 1) ? gU(j - 1, k, col) : T(0);
      nU1ic = j1Int ? gU(j + 1, k, ic1) : T(0);
      nU1id = j1Int ? gU(j + 1, k, id1) : T(0);
    }
  };
  // level k into LDS buffer k & 1, sigma-dot of its lower half level into ring slot (k + 1) % 3
  auto commit = [&](int k) {
    if (!act) return;
    const int bs = k & 1, sn = (k + 1) % 3;
    const C dsg = g.dsig[k];
    const C sh = (k + 1 < nz) ? g.sigh[k + 1] : 0.0;
    if (sdr) {
      S0 += div0(k, nUic, nUid, nV, nVm) * dsg;
      if (d1) S1 += div1(k, nU1ic, nU1id, nV, nV1) * dsg;
      sd0c = sd0n;
      sd1c = sd1n;
      sd0n = 0;
      sd1n = 0;
      if (k + 1 < nz) {
        sd0n = (sh * Pi0 - S0) * rP0sq;
        if (d1) sd1n = (sh * Pi1 - S1) * rP1sq;
      }
    }
    SB(bs, BF, sl) = nF;
    SB(bs, BU, sl) = nU;
    const T u0 = nU * rPU0;
    SB(bs, Bu0, sl) = u0;
    if (hasV) {
      SB(bs, BV, sl) = nV;
      SB(bs, Bvt0, sl) = nV * rPV0 * svj;
      SB(bs, Buv, sl) = T(0.5) * (u0 + nU1 * rPU1);
    }
    if (j >= 1) SB(bs, Bvtm, sl) = nVm * rPVm * svm;
    SD(sn, sl) = (T)sd0n;
    cVm = nVm; cU1 = nU1; cV1 = nV1; cFn = nFn; cFs = nFs; cUs = nUs;
  };

  fetch(0);
  commit(0);
  if (act) SD(0, sl) = T(0);   // half level 0
  __syncthreads();

  const C cc = g.a * g.dlam / (2.0 * g.acap);
  const T rdx2 = T(0.5) * rdx;
  const T rdy2 = T(0.5) * rdyS;
  const int Mv = hasV ? g.Mv[j] : 1, nv = (Mv + 1) / 2;
  const T rdxv2 = hasV ? (T)(1.0 / (2.0 * (double)Mv * g.a * g.sv[j] * g.dlam)) : T(0);
  const T rdyv2 = hasV ? (T)(1.0 / (2.0 * g.a * g.sv[j] * g.dth)) : T(0);
  // wide tiles: the owned column's leap neighbours (i+n-1, i-n, i+n, i+1-n, i+-M, and on the V row
  // i+nv-1, i-nv, i+-Mv) and the level-invariant 1/P^U factors that form u there
  int wcol[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  T wfac[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if constexpr (WIDE) {
    if (own) {
      auto cwr = [&](int o) { return ((col + o) % nx + nx) % nx; };
      auto rp0 = [&](int c) -> T { return isPole ? T(0) : T(2) / (Prow(j, c) + Prow(j, up1(c))); };
      auto rp1 = [&](int c) -> T { return j1Int ? T(2) / (Prow(j + 1, c) + Prow(j + 1, up1(c))) : T(0); };
      const int offs[10] = {nj - 1, -nj, nj, 1 - nj, Mj, -Mj, nv - 1, -nv, Mv, -Mv};
      for (int q = 0; q < 10; ++q) wcol[q] = cwr(offs[q]);
      for (int q = 0; q < 4; ++q) wfac[q] = rp0(wcol[q]);
      wfac[4] = rp0(wcol[6]);
      wfac[5] = rp1(wcol[6]);
      wfac[6] = rp0(wcol[7]);
      wfac[7] = rp1(wcol[7]);
    }
  }
  T pF = 0, pU = 0, pV = 0;   // the owned column's level k-1 values
  const unsigned oc = (unsigned)col;
  // wide tiles: the owned column's leap operands and base values of a level (with WPF those of the
  // next level, fetched while the current one is computed: a wide launch's few workgroups cannot
  // hide a load's latency)
  T wU0 = 0, wU1 = 0, wU2 = 0, wU3 = 0, wF4 = 0, wF5 = 0, wU4 = 0, wU5 = 0;
  T wUa6 = 0, wUa7 = 0, wUb6 = 0, wUb7 = 0, wV8 = 0, wV9 = 0, wbF = 0, wbU = 0, wbV = 0;
  auto wfetch = [&](int k) {
    if (!own) return;
    const unsigned lo = (unsigned)j * row3 + (unsigned)(k * nx);
    if (!isPole) {
      wU0 = gU(j, k, wcol[0]);
      wU1 = gU(j, k, wcol[1]);
      wU2 = gU(j, k, wcol[2]);
      wU3 = gU(j, k, wcol[3]);
      wF4 = gF(j, k, wcol[4]);
      wF5 = gF(j, k, wcol[5]);
      wU4 = gU(j, k, wcol[4]);
      wU5 = gU(j, k, wcol[5]);
      wbF = ldg(A.bF, lo + oc);
      wbU = ldg(A.bU, lo + oc);
    }
    if (hasV) {
      wUa6 = isPole ? T(0) : gU(j, k, wcol[6]);
      wUa7 = isPole ? T(0) : gU(j, k, wcol[7]);
      wUb6 = j1Int ? gU(j + 1, k, wcol[6]) : T(0);
      wUb7 = j1Int ? gU(j + 1, k, wcol[7]) : T(0);
      wV8 = gV(j, k, wcol[8]);
      wV9 = gV(j, k, wcol[9]);
      wbV = ldg(A.bV, lo + oc);
    }
  };
  if constexpr (WPF) wfetch(0);
#pragma unroll 1
  for (int k = 0; k < nz; ++k) {
    const bool more = k + 1 < nz;
    const T cF = nF, cU = nU, cV = nV;   // level k (the fetch below moves to level k+1)
    T baseF = 0, baseU = 0, baseV = 0;
    const unsigned lo = (unsigned)j * row3 + (unsigned)(k * nx);
    // wide tiles with WPF: this level's prefetched operands (the fetch below moves to level k+1)
    const T xU0 = wU0, xU1 = wU1, xU2 = wU2, xU3 = wU3, xF4 = wF4, xF5 = wF5, xU4 = wU4, xU5 = wU5;
    const T xUa6 = wUa6, xUa7 = wUa7, xUb6 = wUb6, xUb7 = wUb7, xV8 = wV8, xV9 = wV9;
    if constexpr (WPF) {
      baseF = wbF;
      baseU = wbU;
      baseV = wbV;
      if (more) wfetch(k + 1);
    } else if (own) {
      if (!isPole) {
        baseF = ldg(A.bF, lo + oc);
        baseU = ldg(A.bU, lo + oc);
      }
      if (hasV) baseV = ldg(A.bV, lo + oc);
    }
    if (more) fetch(k + 1);
    const C dsg = g.dsig[k], r2d = 1.0 / (2.0 * dsg);
    const int bs = k & 1, st = k % 3, sb = (k + 1) % 3;
    // the level-k values at the owned column's leap neighbours: LDS slots (band tiles), or formed from
    // global memory with the level-invariant factors taken before the loop (wide tiles; the same
    // statements as commit's, so that both forms round and contract alike)
    T u0IC = 0, u0ID = 0, u0PA = 0, u0PB = 0, FPM = 0, FMM = 0, UPM = 0, UMM = 0;
    T uvQA = 0, uvQB = 0, VVP = 0, VVM = 0;
    if (own) {
      if constexpr (WPF) {
        auto wuv = [&](T Uc, T U1c, T rp0, T rp1) -> T {
          const T u0 = Uc * rp0;
          return T(0.5) * (u0 + U1c * rp1);
        };
        if (!isPole) {
          u0IC = xU0 * wfac[0];
          u0ID = xU1 * wfac[1];
          u0PA = xU2 * wfac[2];
          u0PB = xU3 * wfac[3];
          FPM = xF4;
          FMM = xF5;
          UPM = xU4;
          UMM = xU5;
        }
        if (hasV) {
          uvQA = wuv(xUa6, xUb6, wfac[4], wfac[5]);
          uvQB = wuv(xUa7, xUb7, wfac[6], wfac[7]);
          VVP = xV8;
          VVM = xV9;
        }
      } else if constexpr (WIDE) {
        auto wu0 = [&](int c, T rp) -> T {
          const T Uc = isPole ? T(0) : gU(j, k, c);
          const T u0 = Uc * rp;
          return u0;
        };
        auto wuv = [&](int c, T rp0, T rp1) -> T {
          const T u0 = wu0(c, rp0);
          const T U1c = j1Int ? gU(j + 1, k, c) : T(0);
          return T(0.5) * (u0 + U1c * rp1);
        };
        if (!isPole) {
          u0IC = wu0(wcol[0], wfac[0]);
          u0ID = wu0(wcol[1], wfac[1]);
          u0PA = wu0(wcol[2], wfac[2]);
          u0PB = wu0(wcol[3], wfac[3]);
          FPM = gF(j, k, wcol[4]);
          FMM = gF(j, k, wcol[5]);
          UPM = gU(j, k, wcol[4]);
          UMM = gU(j, k, wcol[5]);
        }
        if (hasV) {
          uvQA = wuv(wcol[6], wfac[4], wfac[5]);
          uvQB = wuv(wcol[7], wfac[6], wfac[7]);
          VVP = gV(j, k, wcol[8]);
          VVM = gV(j, k, wcol[9]);
        }
      } else {
        if (!isPole) {
          u0IC = SB(bs, Bu0, sl + nj - 1);
          u0ID = SB(bs, Bu0, sl - nj);
          u0PA = SB(bs, Bu0, sl + nj);
          u0PB = SB(bs, Bu0, sl + 1 - nj);
          FPM = SB(bs, BF, sl + Mj);
          FMM = SB(bs, BF, sl - Mj);
          UPM = SB(bs, BU, sl + Mj);
          UMM = SB(bs, BU, sl - Mj);
        }
        if (hasV) {
          uvQA = SB(bs, Buv, sl + nv - 1);
          uvQB = SB(bs, Buv, sl - nv);
          VVP = SB(bs, BV, sl + Mv);
          VVM = SB(bs, BV, sl - Mv);
        }
      }
    }
    if (own) {
      const int sp = sl + 1;
      if (!isPole) {
        // Phi: the leaped centred difference of u Phi, u at the midpoints
        const T L1 = (u0IC * FPM - u0ID * FMM) * rdx2;
        const T L2 = (SB(bs, Bvt0, sl) * cFn - SB(bs, Bvtm, sl) * cFs) * rdy2;
        C L3 = 0;
        if (more) L3 += sd0n * (C)nF;
        if (k > 0) L3 -= sd0c * (C)pF;
        const C TF = -((C)L1 + (C)L2 + L3 * r2d);
        stg(A.oF, lo + oc, (T)((C)baseF + A.ch * TF));
        // U: the same leap on U points, u averaged to the integer points i+n and i+1-n
        const T ubA = T(0.5) * (u0IC + u0PA);
        const T ubB = T(0.5) * (u0ID + u0PB);
        const T U1v = (ubA * UPM - ubB * UMM) * rdx2;
        const T vtn = T(0.5) * (SB(bs, Bvt0, sl) + SB(bs, Bvt0, sp));
        const T vts = T(0.5) * (SB(bs, Bvtm, sl) + SB(bs, Bvtm, sp));
        const T U2v = (vtn * cU1 - vts * cUs) * rdy2;
        C U3 = 0;
        if (more) U3 += (C)(T(0.5) * (SD(sb, sl) + SD(sb, sp))) * (C)nU;
        if (k > 0) U3 -= (C)(T(0.5) * (SD(st, sl) + SD(st, sp))) * (C)pU;
        const C TU = -((C)U1v + (C)U2v + U3 * r2d);
        stg(A.oU, lo + oc, (T)((C)baseU + A.ch * TU));
      } else {
        const C sgn = (j == 0) ? 1.0 : -1.0;
        const C L2 = sgn * cc * cap0[nz + k];
        C L3 = 0;
        if (more) L3 += sd0n * (C)(T)A.pin[pidx * (nz + 1) + k + 1];
        if (k > 0) L3 -= sd0c * (C)(T)A.pin[pidx * (nz + 1) + k - 1];
        const C TF = -(L2 + L3 * r2d);
        const T val = (T)(A.pbase[pidx * (nz + 1) + k] + A.ch * TF);
        stg(A.oF, lo + oc, val);
        stg(A.oU, lo + oc, T(0));
        if (col == 0) A.pout[pidx * (nz + 1) + k] = (double)val;
      }
      if (hasV) {
        const T L1 = (uvQA * VVP - uvQB * VVM) * rdxv2;
        T L2 = T(0);
        if (j + 1 < ny) L2 += T(0.5) * (SB(bs, Bvt0, sl) + cV1 * rPV1 * sv1) * cV1;
        if (j > 0) L2 -= T(0.5) * (SB(bs, Bvtm, sl) + SB(bs, Bvt0, sl)) * cVm;
        L2 = L2 * rdyv2;
        C L3 = 0;
        if (more) L3 += 0.5 * (sd0n + sd1n) * (C)nV;
        if (k > 0) L3 -= 0.5 * (sd0c + sd1c) * (C)pV;
        const C TV = -((C)L1 + (C)L2 + L3 * r2d);
        stg(A.oV, lo + oc, (T)((C)baseV + A.ch * TV));
      }
    }
    pF = cF;
    pU = cU;
    pV = cV;
    if (more) commit(k + 1);
    __syncthreads();
  }

  // p_s is not advected
  if (own) {
    const size_t i2 = (size_t)j * nx + col;
    if (!isPole) {
      A.oP[i2] = A.bP[i2];
    } else {
      const T val = (T)A.pbase[pidx * (nz + 1) + nz];
      A.oP[i2] = val;
      if (col == 0) A.pout[pidx * (nz + 1) + nz] = (double)val;
    }
  }
}

// FP64 cap sums of the advection stage's input, one block per (level, pole), in the fixed order of
// capsum_level: the flux sum_i P^V V through the V row next to the pole and
// sum_i (V / P^V) sin(theta) Phi of the row next to the pole.
template <typename T>
__device__ void capsum_adv_level(const StageArgs<T>& A, int k, int p) {
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const T p0 = (T)g.p0;
  const int ja = (p == 0) ? 1 : ny - 1, jv = (p == 0) ? 0 : ny - 1;
  const T Pp = tsqrt<T>((T)A.pin[(p == 0 ? 0 : nz + 1) + nz] / p0);
  const T* pV = A.inV + ((size_t)jv * nz + k) * nx;
  const T* pF = A.inF + ((size_t)ja * nz + k) * nx;
  const T svv = (T)g.sv[jv];
  const T* pP = A.inP + (size_t)ja * nx;
  C s1 = 0, s2 = 0;
  const int nt = blockDim.x;
  for (int i0 = threadIdx.x; i0 < nx; i0 += nt * kCapChunk) {
    T psv[kCapChunk], vvv[kCapChunk], fv[kCapChunk];
#pragma unroll
    for (int u = 0; u < kCapChunk; ++u) {
      const int i = i0 + nt * u < nx ? i0 + nt * u : i0;
      psv[u] = pP[i];
      vvv[u] = pV[i];
      fv[u] = pF[i];
    }
#pragma unroll
    for (int u = 0; u < kCapChunk; ++u) {
      if (i0 + nt * u >= nx) break;
      const T pv = T(0.5) * (Pp + tsqrt<T>(psv[u] / p0));
      const T vv = vvv[u];
      s1 += (C)(pv * vv);
      s2 += (C)(vv / pv * svv * fv[u]);
    }
  }
  cap_store(A, k, p, s1, s2);
}

template <typename T>
__global__ void __launch_bounds__(kCapBlock) k_capsum_adv(StageArgs<T> a) {
  capsum_adv_level<T>(a, blockIdx.x, blockIdx.y);
}

// The cap sums of every batched member, for the process of its stage.
template <typename T>
__global__ void __launch_bounds__(kCapBlock) k_capsum_batch(const StageArgs<T>* __restrict__ args, int n) {
  const int m = blockIdx.z;
  if (m >= n) return;
  const StageArgs<T> a = args[m];
  if ((int)blockIdx.x >= a.g.nz) return;
  if (a.process == 0) capsum_level<T>(a, blockIdx.x, blockIdx.y);
  else if (a.process == 1) capsum_adv_level<T>(a, blockIdx.x, blockIdx.y);
}

// Advection stage tiles (after k_capsum_adv): one workgroup per zonal tile.  The main launch takes
// the rows whose halos fit its workgroup as band tiles; the rows next to the poles run as wide tiles
// in a second launch (WIDE) that runs beside it, the two on different streams, so that their larger
// register need does not lower the main launch's occupancy (band tiles alone stay within 128 VGPRs:
// four waves per SIMD).
template <typename T, int MAXB, bool WIDE>
__global__ void __launch_bounds__(MAXB) k_stage_atile(StageArgs<T> a, const AatItem* items) {
  extern __shared__ __align__(16) unsigned char smem[];
  const AatItem it = items[blockIdx.x];
  if (it.j < 0) return;
  if constexpr (WIDE) {
    if (it.hl < 0) {
      advect_tile<T, true>(a, it, smem);
      return;
    }
  }
  advect_tile<T, false>(a, it, smem);
}

// One launch per adaptation stage: one workgroup per zonal tile (the cap sums come from k_capsum).
template <typename T>
__global__ void __launch_bounds__(kFwdTileMaxBlock) k_stage_tile(StageArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const AatItem it = a.tiles[blockIdx.x];
  if (it.j < 0) return;
  adapt_tile<T>(a, it, smem);
}

// Persistent batched stage of one process (one launch each, so that each has its own register
// budget).  Work items: the tiles of every member (item = (member, index into the member's tile table
// of that process)); a workgroup takes items b, b+G, ... and skips those whose member is not at that
// process in this stage.  Every column's arithmetic is that of the single-member launches whatever
// the tiling, so members equal their own steps bit for bit.
template <typename T, int PROC>
__global__ void __launch_bounds__(kBatchMaxBlock) k_stage_batch(const StageArgs<T>* __restrict__ args,
                                                                const int2* __restrict__ items, int nitems) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const int2 it = items[w];
    if (it.x < 0) continue;
    const StageArgs<T> a = args[it.x];
    if (a.process != PROC) continue;
    const AatItem ti = PROC == 0 ? a.tiles[it.y] : a.atiles[it.y];
    if (ti.j < 0) continue;
    if constexpr (PROC == 0) adapt_tile<T>(a, ti, smem);
    else if (ti.hl < 0) advect_tile<T, true, false>(a, ti, smem);
    else advect_tile<T, false>(a, ti, smem);
    __syncthreads();
  }
}

// Pole means of Phi (per level) and p_s, FP64, one wavefront per value.
template <typename T>
__global__ void __launch_bounds__(64) k_pole_prep(int nx, int ny, int nz, const T* F, const T* ps, double* pole) {
  const int v = blockIdx.x;          // 0 .. 2*(nz+1)-1
  const int p = v / (nz + 1), k = v % (nz + 1);
  const int j = (p == 0) ? 0 : ny;
  const T* src = (k < nz) ? F + ((size_t)j * nz + k) * nx : ps + (size_t)j * nx;
  C s = 0;
  for (int i = threadIdx.x; i < nx; i += 64) s += (C)src[i];
  s = wave_sum(s);
  if (threadIdx.x == 0) pole[p * (nz + 1) + k] = s / (double)nx;
}

template <typename T>
__global__ void k_copy(T* __restrict__ d, const T* __restrict__ s, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) d[i] = s[i];
}
template <typename T>
__global__ void k_zero(T* __restrict__ d, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) d[i] = T(0);
}

// Global FP64 sums: per block partials of mass, energy (U^2+V^2+Phi^2 weighted), surface q^2.
// Block r handles scalar row r (and V row r if r < ny); pole rows use their mean.
template <typename T>
__global__ void __launch_bounds__(256) k_diag(GeoDev g, const T* U, const T* V, const T* F, const T* ps, double* part) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int j = blockIdx.x;
  __shared__ double red[3][4];
  const double a2 = g.a * g.a;
  double m = 0, e = 0, es = 0;
  const bool pole = (j == 0 || j == ny);
  if (!pole) {
    const double w = a2 * g.s[j] * g.dth * g.dlam;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
      const double p = (double)ps[(size_t)j * nx + i];
      m += w * p;
      const double q = log(p / g.p0) + g.phis[(size_t)j * nx + i] / (g.rd * g.t0);
      es += w * q * q;
      for (int k = 0; k < nz; ++k) {
        const size_t id = ((size_t)j * nz + k) * nx + i;
        const double uu = (double)U[id], ff = (double)F[id];
        e += w * g.dsig[k] * (uu * uu + ff * ff);
      }
    }
  }
  if (j < ny) {
    const double w = a2 * g.sv[j] * g.dth * g.dlam;
    for (int i = threadIdx.x; i < nx; i += blockDim.x)
      for (int k = 0; k < nz; ++k) {
        const double vv = (double)V[((size_t)j * nz + k) * nx + i];
        e += w * g.dsig[k] * vv * vv;
      }
  }
  // wave partials then block partials in a fixed order
  m = wave_sum(m); e = wave_sum(e); es = wave_sum(es);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  if (ln == 0) { red[0][wv] = m; red[1][wv] = e; red[2][wv] = es; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double M = 0, E = 0, ES = 0;
    for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) { M += red[0][w2]; E += red[1][w2]; ES += red[2][w2]; }
    if (pole) {
      // pole contributions: cap area times the row mean
      double pm = 0, qm;
      for (int i = 0; i < nx; ++i) pm += (double)ps[(size_t)j * nx + i];
      pm /= nx;
      M = g.acap * pm;
      qm = log(pm / g.p0) + g.phis[(size_t)j * nx] / (g.rd * g.t0);
      ES = g.acap * qm * qm;
      double ef = 0;
      for (int k = 0; k < nz; ++k) {
        double fm = 0;
        for (int i = 0; i < nx; ++i) fm += (double)F[((size_t)j * nz + k) * nx + i];
        fm /= nx;
        ef += g.acap * g.dsig[k] * fm * fm;
      }
      E += ef;
    }
    part[3 * j + 0] = M;
    part[3 * j + 1] = E;
    part[3 * j + 2] = ES;
  }
}

// The low-latitude filters (Sec. III-B, Table IV rows 1-2), one zonal row of one level per block,
// in place: the row is read into LDS in FP64, then either the 2-dlam wave is removed (the amplitude
// (1/nx) sum_x (-1)^x F_x is summed in FP64 in a fixed order: strided per-thread sums, a butterfly
// per wavefront, the wavefronts in order) or the 3-point operator F + r (F_{x-1} - 2 F + F_{x+1})
// is applied; results are rounded once to the field precision.
template <typename T>
__global__ void __launch_bounds__(256) k_lowlat(int nx, int nz, const FiltItem* items, T* U, T* V, T* F, T* P) {
  extern __shared__ double frow[];
  __shared__ double red[4];
  const FiltItem it = items[blockIdx.y];
  const int k = blockIdx.x;
  if (it.field == 3 && k > 0) return;
  T* base = it.field == 0 ? U : (it.field == 1 ? V : (it.field == 2 ? F : P));
  T* row = base + (it.field == 3 ? (size_t)it.j * nx : ((size_t)it.j * nz + k) * nx);
  const int t = threadIdx.x;
  for (int i = t; i < nx; i += 256) frow[i] = (double)row[i];
  __syncthreads();
  if (it.r < 0.0) {
    double part = 0;
    for (int i = t; i < nx; i += 256) part += (i & 1) ? -frow[i] : frow[i];
    part = wave_sum(part);
    if ((t & 63) == 0) red[t >> 6] = part;
    __syncthreads();
    const double A = (((red[0] + red[1]) + red[2]) + red[3]) / (double)nx;
    for (int i = t; i < nx; i += 256) row[i] = (T)(frow[i] - ((i & 1) ? -A : A));
  } else {
    const double r = it.r;
    for (int i = t; i < nx; i += 256) {
      const double fm = frow[i == 0 ? nx - 1 : i - 1], fp = frow[i == nx - 1 ? 0 : i + 1];
      row[i] = (T)(frow[i] + r * (fm - 2.0 * frow[i] + fp));
    }
  }
}

// Global sums of the per-row partials of k_diag, in a fixed order (each lane adds its rows in
// ascending order, then a fixed butterfly; lane 0's result is written), so a result never depends
// on timing.  out[0] = mass, out[1] = (p0/2g) sum w dsig (U^2 + V^2 + Phi^2) + (R T0 p0/2g) sum w q^2.
__global__ void __launch_bounds__(64) k_diag_final(GeoDev g, const double* part, int nrows, double* out) {
  double m = 0, e = 0, es = 0;
  for (int j = threadIdx.x; j < nrows; j += 64) {
    m += part[3 * j];
    e += part[3 * j + 1];
    es += part[3 * j + 2];
  }
  m = wave_sum(m);
  e = wave_sum(e);
  es = wave_sum(es);
  if (threadIdx.x == 0) {
    out[0] = m;
    out[1] = g.p0 / (2.0 * g.g) * e + g.rd * g.t0 * g.p0 / (2.0 * g.g) * es;
  }
}

template <typename T>
__global__ void k_nonfinite(const T* __restrict__ x, size_t n, unsigned long long* count) {
  unsigned long long c = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const T v = x[i];
    if (!(v == v) || v - v != T(0)) ++c;
  }
  if (c) atomicAdd(count, c);
}

// Dynamic LDS above 64 KB must be enabled per kernel (CDNA4 has 160 KB per CU).
// The attribute is raised to the CDNA4 maximum once per kernel (so that later launches, also inside a
// stream capture, make no runtime call besides the launch).
template <auto Kernel>
hipError_t allow_lds(size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  static bool done = false;   // one flag per kernel
  if (done) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(Kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess) done = true;
  return e;
}

// An adaptation stage: the cap sums of its input, then the tiles.
template <typename T>
hipError_t launch_adapt_tiles(const StageArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_capsum<T>), dim3(a.g.nz, 2), dim3(kCapBlock), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = adapt_tile_lds(a.tblock, sizeof(T));
  e = allow_lds<k_stage_tile<T>>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_stage_tile<T>), dim3(a.ntiles), dim3(a.tblock), lds, s, a);
  return hipGetLastError();
}

// An advection stage: the pole cap sums of its input, then the tiles: the polar ones first on the
// stage's stream, the band tiles beside them on the side stream (without one, after them on the same
// stream).
template <typename T>
hipError_t launch_advect_tiles(const StageArgs<T>& a, hipStream_t s, const SideLaunch* side) {
  hipLaunchKernelGGL((k_capsum_adv<T>), dim3(a.g.nz, 2), dim3(kCapBlock), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool fork = a.nptiles > 0 && side != nullptr;
  hipStream_t ms = s;   // the stream of the main launch
  if (a.nptiles > 0) {
    // the polar tiles go out first, on the stage's stream, the band tiles beside them on the second
    // stream: a polar workgroup needs more registers per wave than a finished band workgroup frees,
    // so queued behind a full band launch it would start only at that launch's tail
    const size_t plds = advect_tile_lds(a.pblock, sizeof(T));
    if (fork) {
      if ((e = hipEventRecord(side->fork, s)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(side->s, side->fork, 0)) != hipSuccess) return e;
      ms = side->s;
    }
    hipLaunchKernelGGL((k_stage_atile<T, 256, true>), dim3(a.nptiles), dim3(a.pblock), plds, s, a, a.ptiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const size_t lds = advect_tile_lds(a.ablock, sizeof(T));
  if (a.awide) hipLaunchKernelGGL((k_stage_atile<T, 256, true>), dim3(a.natiles), dim3(a.ablock), lds, ms, a, a.atiles);
  else hipLaunchKernelGGL((k_stage_atile<T, 256, false>), dim3(a.natiles), dim3(a.ablock), lds, ms, a, a.atiles);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (fork) {
    if ((e = hipEventRecord(side->join, side->s)) != hipSuccess) return e;
    e = hipStreamWaitEvent(s, side->join, 0);
  }
  return e;
}

}  // namespace

size_t adapt_tile_lds_bytes(int block, int elem) { return adapt_tile_lds(block, elem); }
size_t advect_tile_lds_bytes(int block, int elem) { return advect_tile_lds(block, elem); }

template <typename T>
hipError_t launch_stage(const StageArgs<T>& a, hipStream_t s, const SideLaunch* side) {
  return a.process == 0 ? launch_adapt_tiles<T>(a, s) : launch_advect_tiles<T>(a, s, side);
}

template <typename T>
hipError_t launch_stage_batch(const StageArgs<T>* d_args, int nargs, int max_nz, const int2* d_titems, int ntitems,
                              const int2* d_items, int nitems, int grid, int block, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((k_capsum_batch<T>), dim3(max_nz, 2, nargs), dim3(kCapBlock), 0, s, d_args, nargs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ntitems > 0) {
    if ((e = allow_lds<k_stage_batch<T, 0>>(lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_stage_batch<T, 0>), dim3(grid), dim3(block), lds, s, d_args, d_titems, ntitems);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (nitems > 0) {
    if ((e = allow_lds<k_stage_batch<T, 1>>(lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_stage_batch<T, 1>), dim3(grid), dim3(block), lds, s, d_args, d_items, nitems);
    e = hipGetLastError();
  }
  return e;
}

template <typename T>
hipError_t launch_pole_prep(const GeoDev& g, const T* F, const T* ps, double* pole, hipStream_t s) {
  hipLaunchKernelGGL((k_pole_prep<T>), dim3(2 * (g.nz + 1)), dim3(64), 0, s, g.nx, g.ny, g.nz, F, ps, pole);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_diag(const GeoDev& g, const T* U, const T* V, const T* F, const T* ps, double* partial,
                       double* out, hipStream_t s) {
  hipLaunchKernelGGL((k_diag<T>), dim3(g.ny + 1), dim3(256), 0, s, g, U, V, F, ps, partial);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, g, (const double*)partial, g.ny + 1, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lowlat(const GeoDev& g, const FiltItem* items, int nitems, T* U, T* V, T* F, T* P,
                         hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_lowlat<T>), dim3(g.nz, nitems), dim3(256), sizeof(double) * g.nx, s, g.nx, g.nz, items,
                     U, V, F, P);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_nonfinite(const T* x, size_t n, unsigned long long* count, hipStream_t s) {
  hipLaunchKernelGGL((k_nonfinite<T>), dim3(1024), dim3(256), 0, s, x, n, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy_fill(T* dst, const T* src, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_copy<T>), dim3(2048), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zero(T* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_zero<T>), dim3(2048), dim3(256), 0, s, dst, n);
  return hipGetLastError();
}

#define DYC_INST(T)                                                                                          \
  template hipError_t launch_stage<T>(const StageArgs<T>&, hipStream_t, const SideLaunch*);                 \
  template hipError_t launch_stage_batch<T>(const StageArgs<T>*, int, int, const int2*, int, const int2*, int,   \
                                            int, int, size_t, hipStream_t);                                  \
  template hipError_t launch_pole_prep<T>(const GeoDev&, const T*, const T*, double*, hipStream_t);          \
  template hipError_t launch_diag<T>(const GeoDev&, const T*, const T*, const T*, const T*, double*, double*, \
                                     hipStream_t);                                                           \
  template hipError_t launch_nonfinite<T>(const T*, size_t, unsigned long long*, hipStream_t);               \
  template hipError_t launch_lowlat<T>(const GeoDev&, const FiltItem*, int, T*, T*, T*, T*, hipStream_t);   \
  template hipError_t launch_axpy_fill<T>(T*, const T*, size_t, hipStream_t);                                \
  template hipError_t launch_zero<T>(T*, size_t, hipStream_t);
DYC_INST(float)
DYC_INST(double)
template hipError_t launch_zero<unsigned long long>(unsigned long long*, size_t, hipStream_t);

}  // namespace dyc
