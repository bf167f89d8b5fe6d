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

// Largest workgroup per columns-per-thread: bounds the VGPR budget so that the FP64 column
// sums and one level's loads of every owned column stay in registers (768 threads: 170 VGPRs).
constexpr int max_block(int ni) { return ni <= 2 ? 768 : 512; }
int max_block_for(int nx, int block) { return block <= max_block(columns_per_thread(nx, block)) ? 1 : 0; }

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

// FP64 cap sums of the adaptation stage's input, one block (a wavefront) per (level, pole): the
// flux sum_i P^V V through the V row next to the pole and sum_i (V / P^V) (l_adj - l_pole), in a
// fixed order (lane-strided partial sums, then a butterfly), for the pole rows of adapt_tile.
template <typename T>
__device__ void capsum_level(const StageArgs<T>& A, int k, int p) {
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const T p0 = (T)g.p0;
  const int ja = (p == 0) ? 1 : ny - 1, jva = (p == 0) ? 0 : ny - 1;
  const T pps = (T)A.pin[(p == 0 ? 0 : nz + 1) + nz];
  const T Pp = tsqrt<T>(pps / p0), lp = tlog<T>(pps / p0);
  const T* pV = A.inV + ((size_t)jva * nz + k) * nx;
  C s1 = 0, s2 = 0;
  for (int i = threadIdx.x; i < nx; i += 64) {
    const T psa = A.inP[(size_t)ja * nx + i];
    const T Pa = tsqrt<T>(psa / p0), La = tlog<T>(psa / p0);
    const T pv = T(0.5) * (Pp + Pa);
    const T vv = pV[i];
    s1 += (C)(pv * vv);
    s2 += (C)((vv / pv) * (p == 0 ? (La - lp) : (lp - La)));
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (threadIdx.x == 0) {
    A.cap[p * 2 * nz + k] = s1;
    A.cap[p * 2 * nz + nz + k] = s2;
  }
}

template <typename T>
__global__ void __launch_bounds__(64) k_capsum(StageArgs<T> a) {
  capsum_level<T>(a, blockIdx.x, blockIdx.y);
}

// The cap sums of every batched member whose stage is an adaptation stage.
template <typename T>
__global__ void __launch_bounds__(64) k_capsum_batch(const StageArgs<T>* __restrict__ args, int n) {
  const int m = blockIdx.z;
  if (m >= n) return;
  const StageArgs<T> a = args[m];
  if (a.process != 0 || (int)blockIdx.x >= a.g.nz) return;
  capsum_level<T>(a, blockIdx.x, blockIdx.y);
}

// ----------------------------------------------------------------------------------------------
// Advection: out = base - ch * L(in), L in the IAP skew form, zonal part leaped
// ----------------------------------------------------------------------------------------------
// LDS: P rows j and j+1; per level the rows MU(j+1), u(j), u on the V row, Phi(j), U(j), V(j+1/2),
// v sin(theta) on V rows j-1/2 and j+1/2, and sigma-dot of row j at two half levels.  The first
// pass (column totals Pi) reads leap neighbours straight from global memory, without barriers.
template <typename T, int NI>
__device__ void advect_row(const StageArgs<T>& A, const int j, unsigned char* smem) {
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int B = blockDim.x, t = threadIdx.x;
  T* sP0 = reinterpret_cast<T*>(smem);    // P row j
  T* sP1 = sP0 + nx;                       // P row j+1 (south pole WG: row ny-1)
  T* sMU1 = sP1 + nx;                      // MU row j+1 at level k
  T* su0 = sMU1 + nx;                      // u row j
  T* suv = su0 + nx;                       // u averaged to V row j+1/2
  T* sF = suv + nx;                        // Phi row j
  T* sU = sF + nx;                         // U row j
  T* sV = sU + nx;                         // V row j
  T* svtm = sV + nx;                       // v sin(theta) on V row j-1
  T* svt0 = svtm + nx;                     // v sin(theta) on V row j
  T* sSd = svt0 + nx;                      // sigma-dot row j at two half levels [2][nx]
  double* sCap = reinterpret_cast<double*>(smem + ((12 * nx * sizeof(T) + 15) & ~size_t(15)));  // [2][nz]

  const bool isPole = (j == 0 || j == ny);
  const bool hasV = (j < ny);
  const bool j1Pole = (j + 1 == ny);
  const bool j1Int = (j + 1 >= 1 && j + 1 <= ny - 1);
  const int pidx = (j == 0) ? 0 : 1;
  const T p0 = (T)g.p0;
  const size_t row3 = (size_t)nz * nx;

  auto psA = [&](int jr, int i) -> T {
    if (jr == 0) return (T)A.pin[nz];
    if (jr == ny) return (T)A.pin[(nz + 1) + nz];
    return A.inP[(size_t)jr * nx + i];
  };
  auto FA = [&](int jr, int k, int i) -> T {
    if (jr == 0) return (T)A.pin[k];
    if (jr == ny) return (T)A.pin[(nz + 1) + k];
    return A.inF[(size_t)jr * row3 + (size_t)k * nx + i];
  };

  const int ja = (j == 0) ? 1 : ny - 1;   // row next to a pole
  for (int c = 0; c < NI; ++c) {
    const int i = t + c * B;
    if (i < nx) {
      sP0[i] = tsqrt<T>(psA(j, i) / p0);
      sP1[i] = tsqrt<T>(psA(hasV ? j + 1 : ja, i) / p0);
      sSd[i] = T(0);
      sSd[nx + i] = T(0);
    }
  }
  __syncthreads();

  // pole caps of every level (FP64, wavefront 0): cap divergence of the pole row (j pole) or of
  // the south pole seen from row ny-1, and the cap flux of Phi for a pole row
  if ((isPole || (hasV && j1Pole)) && t < 64) {
    const int jv = (j == 0) ? 0 : ny - 1;
    for (int k = 0; k < nz; ++k) {
      const T* pV = A.inV + (size_t)jv * row3 + (size_t)k * nx;
      C s1 = 0, s2 = 0;
      for (int i = t; i < nx; i += 64) {
        const T pv = T(0.5) * (sP0[i] + sP1[i]);
        const T vv = pV[i];
        s1 += (C)(pv * vv);
        if (isPole) s2 += (C)(vv / pv * (T)g.sv[jv] * FA(ja, k, i));
      }
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      if (t == 0) { sCap[k] = s1; sCap[nz + k] = s2; }
    }
  }
  __syncthreads();

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

  // per-column constants
  int ip1[NI], ic[NI], id[NI], ic1[NI], id1[NI];
  T PUc[NI], PUd[NI], rPU0[NI], rPU1[NI], PVm[NI], PV0[NI], PV1[NI], rPVm[NI], rPV0[NI], rPV1[NI];
  C rP0sq[NI], rP1sq[NI], Pi0[NI], Pi1[NI], S0[NI], S1[NI], sd0c[NI], sd1c[NI];
#pragma unroll
  for (int c = 0; c < NI; ++c) {
    const int i = t + c * B;
    const int ii = i < nx ? i : 0;
    ip1[c] = wrp(ii + 1, nx);
    ic[c] = wrp(ii + nj - 1, nx); id[c] = wrp(ii - nj, nx);
    ic1[c] = wrp(ii + nj1 - 1, nx); id1[c] = wrp(ii - nj1, nx);
    const T P0 = sP0[ii], P1 = sP1[ii];
    rP0sq[c] = 1.0 / ((C)P0 * (C)P0);
    rP1sq[c] = hasV ? 1.0 / ((C)P1 * (C)P1) : 0.0;
    PUc[c] = T(0.5) * (sP0[ic[c]] + sP0[wrp(ic[c] + 1, nx)]);
    PUd[c] = T(0.5) * (sP0[id[c]] + sP0[wrp(id[c] + 1, nx)]);
    rPU0[c] = isPole ? T(0) : T(2) / (P0 + sP0[ip1[c]]);
    rPU1[c] = j1Int ? T(2) / (P1 + sP1[ip1[c]]) : T(0);
    PVm[c] = PV0[c] = PV1[c] = rPVm[c] = rPV0[c] = rPV1[c] = T(1);
    if (hasV) { PV0[c] = T(0.5) * (P0 + P1); rPV0[c] = T(1) / PV0[c]; }
    if (j >= 1) { PVm[c] = T(0.5) * (tsqrt<T>(psA(j - 1, ii) / p0) + P0); rPVm[c] = T(1) / PVm[c]; }
    if (j + 2 <= ny) { PV1[c] = T(0.5) * (P1 + tsqrt<T>(psA(j + 2, ii) / p0)); rPV1[c] = T(1) / PV1[c]; }
    Pi0[c] = Pi1[c] = S0[c] = S1[c] = sd0c[c] = sd1c[c] = 0;
  }
  // MU of row j+1 at leap positions comes from LDS in pass B; in pass A from global
  T PU1c[NI], PU1d[NI];
#pragma unroll
  for (int c = 0; c < NI; ++c) {
    PU1c[c] = j1Int ? T(0.5) * (sP1[ic1[c]] + sP1[wrp(ic1[c] + 1, nx)]) : T(0);
    PU1d[c] = j1Int ? T(0.5) * (sP1[id1[c]] + sP1[wrp(id1[c] + 1, nx)]) : T(0);
  }

  // ---- pass A: column totals Pi for rows j and j+1 (no LDS, no barriers)
#pragma unroll 1
  for (int k = 0; k < nz; ++k) {
    const size_t lev = (size_t)k * nx;
    const T* pU0 = isPole ? nullptr : A.inU + (size_t)j * row3 + lev;
    const T* pU1 = j1Int ? A.inU + (size_t)(j + 1) * row3 + lev : nullptr;
    const T* pV0 = hasV ? A.inV + (size_t)j * row3 + lev : nullptr;
    const T* pVm = (j >= 1) ? A.inV + (size_t)(j - 1) * row3 + lev : nullptr;
    const T* pV1 = (j + 1 < ny) ? A.inV + (size_t)(j + 1) * row3 + lev : nullptr;
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      if (i >= nx) continue;
      const T Vj = pV0 ? pV0[i] : T(0);
      C D0, D1 = 0;
      if (isPole) {
        D0 = capD0 * sCap[k];
      } else {
        D0 = (C)((PUc[c] * pU0[ic[c]] - PUd[c] * pU0[id[c]]) * rdx +
                 (svj * (PV0[c] * Vj) - svm * (PVm[c] * pVm[i])) * rdyS);
      }
      if (hasV) {
        if (j1Pole) D1 = capD1 * sCap[k];
        else
          D1 = (C)((PU1c[c] * pU1[ic1[c]] - PU1d[c] * pU1[id1[c]]) * rdx1 +
                   (sv1 * (PV1[c] * pV1[i]) - svj * (PV0[c] * Vj)) * rdyS1);
      }
      Pi0[c] += D0 * g.dsig[k];
      Pi1[c] += D1 * g.dsig[k];
    }
  }

  // ---- pass B
  const C cc = g.a * g.dlam / (2.0 * g.acap);
  const T rdx2 = T(0.5) * rdx;
  const T rdy2 = T(0.5) * rdyS;
  const int Mv = hasV ? g.Mv[j] : 1, nv = (Mv + 1) / 2;
  const T rdxv2 = hasV ? (T)(1.0 / (2.0 * (double)Mv * g.a * g.sv[j] * g.dlam)) : T(0);
  const T rdyv2 = hasV ? (T)(1.0 / (2.0 * g.a * g.sv[j] * g.dth)) : T(0);
  for (int k = 0; k < nz; ++k) {
    const C dsg = g.dsig[k], r2d = 1.0 / (2.0 * dsg);
    const int par = k & 1, parn = (k + 1) & 1;
    const size_t lev = (size_t)k * nx;
    const T* pU0 = isPole ? nullptr : A.inU + (size_t)j * row3 + lev;
    const T* pU1 = j1Int ? A.inU + (size_t)(j + 1) * row3 + lev : nullptr;
    const T* pV0 = hasV ? A.inV + (size_t)j * row3 + lev : nullptr;
    const T* pVm = (j >= 1) ? A.inV + (size_t)(j - 1) * row3 + lev : nullptr;
    const T* pV1 = (j + 1 < ny) ? A.inV + (size_t)(j + 1) * row3 + lev : nullptr;
    // phase 1: loads of this level; LDS rows
    T Vj[NI], Vm[NI], V1[NI], Fn[NI], Fs[NI], Un[NI], Us[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      Vj[c] = Vm[c] = V1[c] = Fn[c] = Fs[c] = Un[c] = Us[c] = T(0);
      if (i < nx) {
        const T Fj = FA(j, k, i);
        const T Uj = pU0 ? pU0[i] : T(0);
        sF[i] = Fj;
        sU[i] = Uj;
        const T u0 = Uj * rPU0[c];
        su0[i] = u0;
        const T U1 = pU1 ? pU1[i] : T(0);
        if (j1Int) sMU1[i] = T(0.5) * (sP1[i] + sP1[ip1[c]]) * U1;
        if (hasV) {
          Vj[c] = pV0[i];
          sV[i] = Vj[c];
          svt0[i] = Vj[c] * rPV0[c] * svj;
          suv[i] = T(0.5) * (u0 + U1 * rPU1[c]);
        }
        if (j >= 1) {
          Vm[c] = pVm[i];
          svtm[i] = Vm[c] * rPVm[c] * svm;
        }
        if (pV1) V1[c] = pV1[i];
        if (!isPole) {
          Fn[c] = FA(j + 1, k, i);
          Fs[c] = FA(j - 1, k, i);
          Un[c] = U1;
          Us[c] = (j - 1 >= 1) ? A.inU[(size_t)(j - 1) * row3 + lev + i] : T(0);
        }
      }
    }
    __syncthreads();
    C sd0n[NI], sd1n[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      C D0 = 0, D1 = 0;
      if (i < nx) {
        if (isPole) {
          D0 = capD0 * sCap[k];
        } else {
          D0 = (C)((PUc[c] * sU[ic[c]] - PUd[c] * sU[id[c]]) * rdx +
                   (svj * (PV0[c] * Vj[c]) - svm * (PVm[c] * Vm[c])) * rdyS);
        }
        if (hasV) {
          if (j1Pole) D1 = capD1 * sCap[k];
          else
            D1 = (C)((sMU1[ic1[c]] - sMU1[id1[c]]) * rdx1 + (sv1 * (PV1[c] * V1[c]) - svj * (PV0[c] * Vj[c])) * rdyS1);
        }
      }
      S0[c] += D0 * dsg;
      S1[c] += D1 * dsg;
      sd0n[c] = 0; sd1n[c] = 0;
      if (k + 1 < nz && i < nx) {
        const C sh = g.sigh[k + 1];
        sd0n[c] = (sh * Pi0[c] - S0[c]) * rP0sq[c];
        if (hasV) sd1n[c] = (sh * Pi1[c] - S1[c]) * rP1sq[c];
      }
      if (i < nx) sSd[parn * nx + i] = (T)sd0n[c];
    }
    __syncthreads();

    if (!isPole) {
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i >= nx) continue;
        const size_t idx = (size_t)j * row3 + lev + i;
        const int pM = wrp(i + Mj, nx), mM = wrp(i - Mj, nx);
        // Phi: zonal (x+1,x-1) -> (x+2N-1, x-2N+1), u at the midpoints
        const T L1 = (su0[ic[c]] * sF[pM] - su0[id[c]] * sF[mM]) * rdx2;
        const T L2 = (svt0[i] * Fn[c] - svtm[i] * Fs[c]) * rdy2;
        C L3 = 0;
        if (k + 1 < nz) L3 += sd0n[c] * (C)A.inF[idx + nx];
        if (k > 0) L3 -= sd0c[c] * (C)A.inF[idx - nx];
        const C TF = -((C)L1 + (C)L2 + L3 * r2d);
        A.oF[idx] = (T)((C)A.bF[idx] + A.ch * TF);
        // U: same leap on U points with u averaged to the integer points i+n and i+1-n
        const int pA = wrp(i + nj, nx), pB = wrp(i + 1 - nj, nx);
        const T ubA = T(0.5) * (su0[ic[c]] + su0[pA]);
        const T ubB = T(0.5) * (su0[id[c]] + su0[pB]);
        const T U1v = (ubA * sU[pM] - ubB * sU[mM]) * rdx2;
        const int ip = ip1[c];
        const T vtn = T(0.5) * (svt0[i] + svt0[ip]);
        const T vts = T(0.5) * (svtm[i] + svtm[ip]);
        const T U2v = (vtn * Un[c] - vts * Us[c]) * rdy2;
        C U3 = 0;
        if (k + 1 < nz) U3 += (C)(T(0.5) * (sSd[parn * nx + i] + sSd[parn * nx + ip])) * (C)A.inU[idx + nx];
        if (k > 0) U3 -= (C)(T(0.5) * (sSd[par * nx + i] + sSd[par * nx + ip])) * (C)A.inU[idx - nx];
        const C TU = -((C)U1v + (C)U2v + U3 * r2d);
        A.oU[idx] = (T)((C)A.bU[idx] + A.ch * TU);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      const C sgn = (j == 0) ? 1.0 : -1.0;
      const C L2 = sgn * cc * sCap[nz + k];
      C L3 = 0;
      if (k + 1 < nz) L3 += sd0n[0] * (C)FA(j, k + 1, 0);
      if (k > 0) L3 -= sd0c[0] * (C)FA(j, k - 1, 0);
      const C TF = -(L2 + L3 * r2d);
      const T val = (T)(A.pbase[pidx * (nz + 1) + k] + A.ch * TF);
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i < nx) {
          const size_t idx = (size_t)j * row3 + lev + i;
          A.oF[idx] = val;
          A.oU[idx] = T(0);
        }
      }
      if (t == 0) A.pout[pidx * (nz + 1) + k] = (double)val;
    }

    if (hasV) {
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i >= nx) continue;
        const size_t idv = (size_t)j * row3 + lev + i;
        const T L1 = (suv[wrp(i + nv - 1, nx)] * sV[wrp(i + Mv, nx)] - suv[wrp(i - nv, nx)] * sV[wrp(i - Mv, nx)]) * rdxv2;
        T L2 = T(0);
        if (j + 1 < ny) L2 += T(0.5) * (svt0[i] + V1[c] * rPV1[c] * sv1) * V1[c];
        if (j > 0) L2 -= T(0.5) * (svtm[i] + svt0[i]) * Vm[c];
        L2 = L2 * rdyv2;
        C L3 = 0;
        if (k + 1 < nz) L3 += 0.5 * (sd0n[c] + sd1n[c]) * (C)A.inV[idv + nx];
        if (k > 0) L3 -= 0.5 * (sd0c[c] + sd1c[c]) * (C)A.inV[idv - nx];
        const C TV = -((C)L1 + (C)L2 + L3 * r2d);
        A.oV[idv] = (T)((C)A.bV[idv] + A.ch * TV);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int c = 0; c < NI; ++c) { sd0c[c] = sd0n[c]; sd1c[c] = sd1n[c]; }
    __syncthreads();
  }

  // p_s is not advected
  if (!isPole) {
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      if (i < nx) A.oP[(size_t)j * nx + i] = A.bP[(size_t)j * nx + i];
    }
  } else {
    const T val = (T)A.pbase[pidx * (nz + 1) + nz];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      if (i < nx) A.oP[(size_t)j * nx + i] = val;
    }
    if (t == 0) A.pout[pidx * (nz + 1) + nz] = (double)val;
  }
}

// Advection, software-pipelined (the same LDS limit as the adaptation).  LDS: the P rows j and j+1, the reciprocal
// U-point averages of P on rows j and j+1, the V-point averages of P (and their reciprocals) on
// V rows j-1/2, j+1/2, j+3/2, the per-level rows (Phi, U, u of row j, V, the u average on the V
// row, v sin(theta) on V rows j+-1/2) double-buffered, and sigma-dot of row j in a ring of three
// half levels.  Level k+1 (own columns, the leap gathers of U that its divergence needs, and the
// base values) is fetched while level k is computed; the vertical neighbours come from a rolling
// register window, so each level is read from memory once.  One barrier per level.
constexpr int kAdvectPipeRows2D = 10, kAdvectPipeRowsLev = 7;
__host__ __device__ constexpr size_t advect_pipe_lds(int nx, int elem) {
  return (((size_t)(kAdvectPipeRows2D + 2 * kAdvectPipeRowsLev + 3) * nx * elem + 15) & ~size_t(15)) +
         2 * 128 * sizeof(double);
}
__host__ __device__ constexpr bool advect_pipe_ok(int nx, int elem) { return advect_pipe_lds(nx, elem) <= 160 * 1024; }

template <typename T, int NI>
__device__ void advect_row_pipe(const StageArgs<T>& A, const int j, unsigned char* smem) {
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int B = blockDim.x;
  int t = threadIdx.x;   // re-made opaque every level: column indices are recomputed, not held
  // LDS cells column-major, 27 words per column: the 10 2D rows, the two buffers of 7 level rows
  // and the 3-slot sigma-dot ring; one address per column index serves every row (the row is an
  // immediate offset) and consecutive lanes stride 27 words (no bank conflicts)
  constexpr int RS = kAdvectPipeRows2D + 2 * kAdvectPipeRowsLev + 3;
  T* r = reinterpret_cast<T*>(smem);
  auto S2 = [&](int row, int col) -> T& { return r[col * RS + row]; };
  auto SB = [&](int bsel, int row, int col) -> T& {
    return r[col * RS + kAdvectPipeRows2D + bsel * kAdvectPipeRowsLev + row];
  };
  auto SD = [&](int slot, int col) -> T& { return r[col * RS + kAdvectPipeRows2D + 2 * kAdvectPipeRowsLev + slot]; };
  enum { RP0, RP1, RrPU0, RrPU1, RPV0, RPVm, RPV1, RrPV0, RrPVm, RrPV1 };
  enum { BF, BU, Bu0, BV, Buv, Bvt0, Bvtm };
  double* sCap = reinterpret_cast<double*>(
      smem + ((((size_t)kAdvectPipeRows2D + 2 * kAdvectPipeRowsLev + 3) * nx * sizeof(T) + 15) & ~size_t(15)));

  const bool isPole = (j == 0 || j == ny);
  const bool hasV = (j < ny);
  const bool j1Pole = (j + 1 == ny);
  const bool j1Int = (j + 1 >= 1 && j + 1 <= ny - 1);
  const int pidx = (j == 0) ? 0 : 1;
  const T p0 = (T)g.p0;
  const size_t row3 = (size_t)nz * nx;
  auto psA = [&](int jr, int i) -> T {
    if (jr == 0) return (T)A.pin[nz];
    if (jr == ny) return (T)A.pin[(nz + 1) + nz];
    return A.inP[(size_t)jr * nx + i];
  };
  auto FA = [&](int jr, int k, int i) -> T {
    if (jr == 0) return (T)A.pin[k];
    if (jr == ny) return (T)A.pin[(nz + 1) + k];
    return A.inF[(size_t)jr * row3 + (size_t)k * nx + i];
  };

  // ---- 2D rows
  const int ja = (j == 0) ? 1 : ny - 1;   // row next to a pole
  for (int c = 0; c < NI; ++c) {
    const int i = t + c * B;
    if (i < nx) {
      const T P0 = tsqrt<T>(psA(j, i) / p0);
      const T P1 = tsqrt<T>(psA(hasV ? j + 1 : ja, i) / p0);
      S2(RP0, i) = P0;
      S2(RP1, i) = P1;
      T PV0 = T(1), PVm = T(1), PV1 = T(1);
      if (hasV) PV0 = T(0.5) * (P0 + P1);
      if (j >= 1) PVm = T(0.5) * (tsqrt<T>(psA(j - 1, i) / p0) + P0);
      if (j + 2 <= ny) PV1 = T(0.5) * (P1 + tsqrt<T>(psA(j + 2, i) / p0));
      S2(RPV0, i) = PV0; S2(RPVm, i) = PVm; S2(RPV1, i) = PV1;
      S2(RrPV0, i) = T(1) / PV0; S2(RrPVm, i) = T(1) / PVm; S2(RrPV1, i) = T(1) / PV1;
      SD(0, i) = T(0);   // half level 0
    }
  }
  __syncthreads();
  if ((isPole || (hasV && j1Pole)) && t < 64) {
    const int jv = (j == 0) ? 0 : ny - 1;
    for (int k = 0; k < nz; ++k) {
      const T* pV = A.inV + (size_t)jv * row3 + (size_t)k * nx;
      C s1 = 0, s2 = 0;
      for (int i = t; i < nx; i += 64) {
        const T pv = T(0.5) * (S2(RP0, i) + S2(RP1, i));
        const T vv = pV[i];
        s1 += (C)(pv * vv);
        if (isPole) s2 += (C)(vv / pv * (T)g.sv[jv] * FA(ja, k, i));
      }
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      if (t == 0) { sCap[k] = s1; sCap[nz + k] = s2; }
    }
  }
  for (int c = 0; c < NI; ++c) {
    const int i = t + c * B;
    if (i < nx) {
      const int ip = wrp_up(i + 1, nx);
      S2(RrPU0, i) = isPole ? T(0) : T(2) / (S2(RP0, i) + S2(RP0, ip));
      S2(RrPU1, i) = j1Int ? T(2) / (S2(RP1, i) + S2(RP1, ip)) : T(0);
    }
  }

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

  // per-column constants: 1 / P^2 (FP64)
  C rP0sq[NI], rP1sq[NI];
#pragma unroll
  for (int c = 0; c < NI; ++c) {
    const int i = t + c * B;
    const int ii = i < nx ? i : 0;
    rP0sq[c] = 1.0 / ((C)S2(RP0, ii) * (C)S2(RP0, ii));
    rP1sq[c] = hasV ? 1.0 / ((C)S2(RP1, ii) * (C)S2(RP1, ii)) : 0.0;
  }
  __syncthreads();

  // divergence of rows j and j+1 at level k from the owned column's values and leap gathers
  auto div0 = [&](int k, int c, T Uic, T Uid, T Vj, T Vm) -> C {
    if (isPole) return capD0 * sCap[k];
    const int i = t + c * B;
    const int ii = i < nx ? i : 0;
    const int ic = wrp_up(ii + nj - 1, nx), id = wrp_dn(ii - nj, nx);
    const T PUc = T(0.5) * (S2(RP0, ic) + S2(RP0, wrp_up(ic + 1, nx)));
    const T PUd = T(0.5) * (S2(RP0, id) + S2(RP0, wrp_up(id + 1, nx)));
    return (C)((PUc * Uic - PUd * Uid) * rdx + (svj * (S2(RPV0, ii) * Vj) - svm * (S2(RPVm, ii) * Vm)) * rdyS);
  };
  auto div1 = [&](int k, int c, T U1ic, T U1id, T Vj, T V1) -> C {
    if (!hasV) return 0.0;
    if (j1Pole) return capD1 * sCap[k];
    const int i = t + c * B;
    const int ii = i < nx ? i : 0;
    const int ic1 = wrp_up(ii + nj1 - 1, nx), id1 = wrp_dn(ii - nj1, nx);
    const T PU1c = T(0.5) * (S2(RP1, ic1) + S2(RP1, wrp_up(ic1 + 1, nx)));
    const T PU1d = T(0.5) * (S2(RP1, id1) + S2(RP1, wrp_up(id1 + 1, nx)));
    return (C)((PU1c * U1ic - PU1d * U1id) * rdx1 + (sv1 * (S2(RPV1, ii) * V1) - svj * (S2(RPV0, ii) * Vj)) * rdyS1);
  };

  // ---- pass A: column totals Pi of rows j and j+1
  C Pi0[NI], Pi1[NI];
#pragma unroll
  for (int c = 0; c < NI; ++c) { Pi0[c] = 0; Pi1[c] = 0; }
  {
    constexpr int KU = 3;
    for (int k0 = 0; k0 < nz; k0 += KU) {
      T a0[KU][NI], a1[KU][NI], a2[KU][NI], a3[KU][NI], a4[KU][NI], a5[KU][NI], a6[KU][NI];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + u < nz ? k0 + u : nz - 1;
        const size_t lo = (size_t)j * row3 + (size_t)k * nx;
        const auto gU0 = urow(A.inU, lo);
        const auto gU1 = urow(A.inU, lo + row3);
        const auto gV0 = urow(A.inV, lo);
        const auto gVm = urow(A.inV, (lo - (j >= 1 ? row3 : 0)));
        const auto gV1 = urow(A.inV, lo + row3);
#pragma unroll
        for (int c = 0; c < NI; ++c) {
          const int i = t + c * B;
          const int ii = i < nx ? i : 0;
          a0[u][c] = isPole ? T(0) : gU0[(unsigned)wrp_up(ii + nj - 1, nx)];
          a1[u][c] = isPole ? T(0) : gU0[(unsigned)wrp_dn(ii - nj, nx)];
          a2[u][c] = j1Int ? gU1[(unsigned)wrp_up(ii + nj1 - 1, nx)] : T(0);
          a3[u][c] = j1Int ? gU1[(unsigned)wrp_dn(ii - nj1, nx)] : T(0);
          a4[u][c] = hasV ? gV0[(unsigned)ii] : T(0);
          a5[u][c] = (j >= 1) ? gVm[(unsigned)ii] : T(0);
          a6[u][c] = (j + 1 < ny) ? gV1[(unsigned)ii] : T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + u;
        if (k < nz) {
          const C dsg = g.dsig[k];
#pragma unroll
          for (int c = 0; c < NI; ++c) {
            Pi0[c] += div0(k, c, a0[u][c], a1[u][c], a4[u][c], a5[u][c]) * dsg;
            Pi1[c] += div1(k, c, a2[u][c], a3[u][c], a4[u][c], a6[u][c]) * dsg;
          }
        }
      }
    }
  }

  // ---- pass B, pipelined over levels
  // next level (fetched one level ahead)
  T nF[NI], nU[NI], nV[NI], nVm[NI], nU1[NI], nV1[NI], nFn[NI], nFs[NI], nUs[NI];
  T nUic[NI], nUid[NI], nU1ic[NI], nU1id[NI];
  // current level (the level above is read back from the other LDS buffer)
  T cVm[NI], cU1[NI], cV1[NI], cFn[NI], cFs[NI], cUs[NI];
  C S0[NI], S1[NI], sd0c[NI], sd0n[NI], sd1c[NI], sd1n[NI];
#pragma unroll
  for (int c = 0; c < NI; ++c) S0[c] = S1[c] = sd0c[c] = sd0n[c] = sd1c[c] = sd1n[c] = 0;

  auto fetch = [&](int k) {
    const size_t lo = (size_t)j * row3 + (size_t)k * nx;
    const auto gF0 = urow(A.inF, lo);
    const auto gU0 = urow(A.inU, lo);
    const auto gV0 = urow(A.inV, lo);
    const auto gVm = urow(A.inV, (lo - (j >= 1 ? row3 : 0)));
    const auto gU1 = urow(A.inU, lo + row3);
    const auto gV1 = urow(A.inV, lo + row3);
    const auto gF1 = urow(A.inF, lo + row3);
    const auto gFs = urow(A.inF, (lo - (j >= 1 ? row3 : 0)));
    const auto gUs = urow(A.inU, (lo - (j >= 1 ? row3 : 0)));
    const T Fp0 = isPole ? (T)A.pin[pidx * (nz + 1) + k] : T(0);
    const T Fn_p = (j + 1 == ny) ? (T)A.pin[(nz + 1) + k] : T(0);
    const T Fs_p = (j - 1 == 0) ? (T)A.pin[k] : T(0);
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      const unsigned ii = i < nx ? (unsigned)i : 0u;
      nF[c] = isPole ? Fp0 : gF0[ii];
      nU[c] = isPole ? T(0) : gU0[ii];
      nV[c] = hasV ? gV0[ii] : T(0);
      nVm[c] = (j >= 1) ? gVm[ii] : T(0);
      nU1[c] = j1Int ? gU1[ii] : T(0);
      nV1[c] = (j + 1 < ny) ? gV1[ii] : T(0);
      nFn[c] = (!isPole && j + 1 < ny) ? gF1[ii] : Fn_p;
      nFs[c] = (!isPole && j - 1 >= 1) ? gFs[ii] : Fs_p;
      nUs[c] = (!isPole && j - 1 >= 1) ? gUs[ii] : T(0);
      nUic[c] = isPole ? T(0) : gU0[(unsigned)wrp_up((int)ii + nj - 1, nx)];
      nUid[c] = isPole ? T(0) : gU0[(unsigned)wrp_dn((int)ii - nj, nx)];
      nU1ic[c] = j1Int ? gU1[(unsigned)wrp_up((int)ii + nj1 - 1, nx)] : T(0);
      nU1id[c] = j1Int ? gU1[(unsigned)wrp_dn((int)ii - nj1, nx)] : T(0);
    }
  };
  // level k into LDS buffer k & 1; sigma-dot of its lower half level into slot (k + 1) % 3;
  // then the window moves down one level
  auto commit = [&](int k) {
    const int bs = k & 1, sn = (k + 1) % 3;
    const C dsg = g.dsig[k];
    const C sh = (k + 1 < nz) ? g.sigh[k + 1] : 0.0;
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      const C D0 = div0(k, c, nUic[c], nUid[c], nV[c], nVm[c]);
      const C D1 = div1(k, c, nU1ic[c], nU1id[c], nV[c], nV1[c]);
      S0[c] += D0 * dsg;
      S1[c] += D1 * dsg;
      sd0c[c] = sd0n[c];
      sd1c[c] = sd1n[c];
      sd0n[c] = 0;
      sd1n[c] = 0;
      if (k + 1 < nz) {
        sd0n[c] = (sh * Pi0[c] - S0[c]) * rP0sq[c];
        if (hasV) sd1n[c] = (sh * Pi1[c] - S1[c]) * rP1sq[c];
      }
      if (i < nx) {
        SB(bs, BF, i) = nF[c];
        SB(bs, BU, i) = nU[c];
        const T u0 = nU[c] * S2(RrPU0, i);
        SB(bs, Bu0, i) = u0;
        if (hasV) {
          SB(bs, BV, i) = nV[c];
          SB(bs, Bvt0, i) = nV[c] * S2(RrPV0, i) * svj;
          SB(bs, Buv, i) = T(0.5) * (u0 + nU1[c] * S2(RrPU1, i));
        }
        if (j >= 1) SB(bs, Bvtm, i) = nVm[c] * S2(RrPVm, i) * svm;
        SD(sn, i) = (T)sd0n[c];
      }
      cVm[c] = nVm[c]; cU1[c] = nU1[c]; cV1[c] = nV1[c];
      cFn[c] = nFn[c]; cFs[c] = nFs[c]; cUs[c] = nUs[c];
    }
  };

  fetch(0);
  commit(0);
  __syncthreads();

  const C cc = g.a * g.dlam / (2.0 * g.acap);
  const T rdx2 = T(0.5) * rdx;
  const T rdy2 = T(0.5) * rdyS;
  const int Mv = hasV ? g.Mv[j] : 1, nv = (Mv + 1) / 2;
  const T rdxv2 = hasV ? (T)(1.0 / (2.0 * (double)Mv * g.a * g.sv[j] * g.dlam)) : T(0);
  const T rdyv2 = hasV ? (T)(1.0 / (2.0 * g.a * g.sv[j] * g.dth)) : T(0);
#pragma unroll 1
  for (int k = 0; k < nz; ++k) {
    asm volatile("" : "+v"(t));
    const bool more = k + 1 < nz;
    if (more) fetch(k + 1);
    const C dsg = g.dsig[k], r2d = 1.0 / (2.0 * dsg);
    // buffer of level k, the other buffer (level k-1, own columns only), sigma-dot slots above and below
    const int bs = k & 1, ob = (k + 1) & 1, st = k % 3, sb = (k + 1) % 3;
    const size_t lo = (size_t)j * row3 + (size_t)k * nx;
    const auto goF = urow(A.oF, lo);
    const auto goU = urow(A.oU, lo);
    const auto goV = urow(A.oV, lo);
    const auto gbF = urow(A.bF, lo);
    const auto gbU = urow(A.bU, lo);
    const auto gbV = urow(A.bV, lo);
    T cbF[NI], cbU[NI], cbV[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      const unsigned ii = i < nx ? (unsigned)i : 0u;
      cbF[c] = isPole ? T(0) : gbF[ii];
      cbU[c] = isPole ? T(0) : gbU[ii];
      cbV[c] = hasV ? gbV[ii] : T(0);
    }

    if (!isPole) {
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i >= nx) continue;
        const int ic = wrp_up(i + nj - 1, nx), id = wrp_dn(i - nj, nx);
        const int pM = wrp_up(i + Mj, nx), mM = wrp_dn(i - Mj, nx);
        // Phi: zonal (x+1, x-1) -> (x+2N-1, x-2N+1) with u at the midpoints
        const T L1 = (SB(bs, Bu0, ic) * SB(bs, BF, pM) - SB(bs, Bu0, id) * SB(bs, BF, mM)) * rdx2;
        const T L2 = (SB(bs, Bvt0, i) * cFn[c] - SB(bs, Bvtm, i) * cFs[c]) * rdy2;
        C L3 = 0;
        if (more) L3 += sd0n[c] * (C)nF[c];
        if (k > 0) L3 -= sd0c[c] * (C)SB(ob, BF, i);
        const C TF = -((C)L1 + (C)L2 + L3 * r2d);
        goF[i] = (T)((C)cbF[c] + A.ch * TF);
        // U: the same leap on U points, u averaged to the integer points i+n and i+1-n
        const int pA = wrp_up(i + nj, nx), pB = wrp_dn(i + 1 - nj, nx);
        const T ubA = T(0.5) * (SB(bs, Bu0, ic) + SB(bs, Bu0, pA));
        const T ubB = T(0.5) * (SB(bs, Bu0, id) + SB(bs, Bu0, pB));
        const T U1v = (ubA * SB(bs, BU, pM) - ubB * SB(bs, BU, mM)) * rdx2;
        const int ip = wrp_up(i + 1, nx);
        const T vtn = T(0.5) * (SB(bs, Bvt0, i) + SB(bs, Bvt0, ip));
        const T vts = T(0.5) * (SB(bs, Bvtm, i) + SB(bs, Bvtm, ip));
        const T U2v = (vtn * cU1[c] - vts * cUs[c]) * rdy2;
        C U3 = 0;
        if (more) U3 += (C)(T(0.5) * (SD(sb, i) + SD(sb, ip))) * (C)nU[c];
        if (k > 0) U3 -= (C)(T(0.5) * (SD(st, i) + SD(st, ip))) * (C)SB(ob, BU, i);
        const C TU = -((C)U1v + (C)U2v + U3 * r2d);
        goU[i] = (T)((C)cbU[c] + A.ch * TU);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      const C sgn = (j == 0) ? 1.0 : -1.0;
      const C L2 = sgn * cc * sCap[nz + k];
      C L3 = 0;
      if (more) L3 += sd0n[0] * (C)FA(j, k + 1, 0);
      if (k > 0) L3 -= sd0c[0] * (C)FA(j, k - 1, 0);
      const C TF = -(L2 + L3 * r2d);
      const T val = (T)(A.pbase[pidx * (nz + 1) + k] + A.ch * TF);
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i < nx) {
          goF[i] = val;
          goU[i] = T(0);
        }
      }
      if (t == 0) A.pout[pidx * (nz + 1) + k] = (double)val;
    }

    if (hasV) {
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i >= nx) continue;
        const T L1 = (SB(bs, Buv, wrp_up(i + nv - 1, nx)) * SB(bs, BV, wrp_up(i + Mv, nx)) - SB(bs, Buv, wrp_dn(i - nv, nx)) * SB(bs, BV, wrp_dn(i - Mv, nx))) * rdxv2;
        T L2 = T(0);
        if (j + 1 < ny) L2 += T(0.5) * (SB(bs, Bvt0, i) + cV1[c] * S2(RrPV1, i) * sv1) * cV1[c];
        if (j > 0) L2 -= T(0.5) * (SB(bs, Bvtm, i) + SB(bs, Bvt0, i)) * cVm[c];
        L2 = L2 * rdyv2;
        C L3 = 0;
        if (more) L3 += 0.5 * (sd0n[c] + sd1n[c]) * (C)nV[c];
        if (k > 0) L3 -= 0.5 * (sd0c[c] + sd1c[c]) * (C)SB(ob, BV, i);
        const C TV = -((C)L1 + (C)L2 + L3 * r2d);
        goV[i] = (T)((C)cbV[c] + A.ch * TV);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (more) commit(k + 1);
    __syncthreads();
  }

  // p_s is not advected
  if (!isPole) {
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      if (i < nx) A.oP[(size_t)j * nx + i] = A.bP[(size_t)j * nx + i];
    }
  } else {
    const T val = (T)A.pbase[pidx * (nz + 1) + nz];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      if (i < nx) A.oP[(size_t)j * nx + i] = val;
    }
    if (t == 0) A.pout[pidx * (nz + 1) + nz] = (double)val;
  }
}

// One launch per advection stage; the form is a template parameter so that the row kernels are
// separate symbols in a profile.  PROC: 1 advection, 3 its pipelined form (rows whose 27 LDS rows fit
// in 160 KB).
template <typename T, int NI, int PROC>
__global__ void __launch_bounds__(max_block(NI)) k_stage(StageArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int j = xcd_row(blockIdx.x, a.g.ny + 1);
  if constexpr (PROC == 3) advect_row_pipe<T, NI>(a, j, smem);
  else advect_row<T, NI>(a, j, smem);
}

// One launch per adaptation stage: one workgroup per zonal tile (the cap sums come from k_capsum).
template <typename T>
__global__ void __launch_bounds__(kFwdTileMaxBlock) k_stage_tile(StageArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const AatItem it = a.tiles[blockIdx.x];
  if (it.j < 0) return;
  adapt_tile<T>(a, it, smem);
}

// Persistent batched stage.  Work items: first the adaptation tiles of every member (tile item =
// (member, index into the member's tile table)), then the advection rows (row item = (member, row));
// a workgroup takes items b, b+G, ... and skips those whose member is not at that process in this
// stage.  PIPE: 1 when every member's advection takes the pipelined form, 0 when none does, 2 mixed.
template <typename T, int NI, int PIPE>
__global__ void __launch_bounds__(max_block(NI)) k_stage_batch(const StageArgs<T>* __restrict__ args,
                                                               const int2* __restrict__ titems, int ntitems,
                                                               const int2* __restrict__ items, int nitems) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int w = blockIdx.x; w < ntitems + nitems; w += gridDim.x) {
    const bool tile = w < ntitems;
    const int2 it = tile ? titems[w] : items[w - ntitems];
    if (it.x < 0) continue;
    const StageArgs<T> a = args[it.x];
    if (tile) {
      if (a.process != 0) continue;
      const AatItem ti = a.tiles[it.y];
      if (ti.j < 0) continue;
      adapt_tile<T>(a, ti, smem);
    } else {
      if (a.process != 1) continue;
      if constexpr (PIPE == 1) advect_row_pipe<T, NI>(a, it.y, smem);
      else if constexpr (PIPE == 0) advect_row<T, NI>(a, it.y, smem);
      else if (advect_pipe_ok(a.g.nx, sizeof(T))) advect_row_pipe<T, NI>(a, it.y, smem);
      else advect_row<T, NI>(a, it.y, smem);
    }
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

template <typename T, int NI>
hipError_t launch_stage_ni(const StageArgs<T>& a, int block, hipStream_t s) {
  const size_t lds = stage_lds_bytes(a.process, a.g.nx, sizeof(T));
  hipError_t e;
  if (advect_pipe_ok(a.g.nx, sizeof(T))) {
    e = allow_lds<k_stage<T, NI, 3>>(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stage<T, NI, 3>), dim3(a.g.ny + 1), dim3(block), lds, s, a);
  } else {
    e = allow_lds<k_stage<T, NI, 1>>(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stage<T, NI, 1>), dim3(a.g.ny + 1), dim3(block), lds, s, a);
  }
  return hipGetLastError();
}

// An adaptation stage: the cap sums of its input, then the tiles.
template <typename T>
hipError_t launch_adapt_tiles(const StageArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_capsum<T>), dim3(a.g.nz, 2), dim3(64), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = adapt_tile_lds(a.tblock, sizeof(T));
  e = allow_lds<k_stage_tile<T>>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_stage_tile<T>), dim3(a.ntiles), dim3(a.tblock), lds, s, a);
  return hipGetLastError();
}

template <typename T, int NI, int PIPE>
hipError_t launch_batch_pipe(const StageArgs<T>* d_args, const int2* d_titems, int ntitems, const int2* d_items,
                             int nitems, int grid, int block, size_t lds, hipStream_t s) {
  hipError_t e = allow_lds<k_stage_batch<T, NI, PIPE>>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_stage_batch<T, NI, PIPE>), dim3(grid), dim3(block), lds, s, d_args, d_titems, ntitems,
                     d_items, nitems);
  return hipGetLastError();
}

template <typename T, int NI>
hipError_t launch_batch_ni(const StageArgs<T>* d_args, const int2* d_titems, int ntitems, const int2* d_items,
                           int nitems, int grid, int block, size_t lds, int pipe, hipStream_t s) {
  if (pipe == 1) return launch_batch_pipe<T, NI, 1>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, s);
  if (pipe == 2) return launch_batch_pipe<T, NI, 2>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, s);
  return launch_batch_pipe<T, NI, 0>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, s);
}

}  // namespace

size_t stage_lds_bytes(int process, int nx, int elem) {
  if (process == 0) return adapt_tile_lds(elem == 4 ? kFwdTileMaxBlock : 704, elem);   // the largest tile block
  if (advect_pipe_ok(nx, elem)) return advect_pipe_lds(nx, elem);
  const size_t rows = 12;
  return ((rows * (size_t)nx * elem + 15) & ~size_t(15)) + 2 * 128 * sizeof(double);
}

int columns_per_thread(int nx, int block) { return (nx + block - 1) / block; }
size_t adapt_tile_lds_bytes(int block, int elem) { return adapt_tile_lds(block, elem); }
int stage_pipelined(int nx, int elem) { return advect_pipe_ok(nx, elem) ? 1 : 0; }

template <typename T>
hipError_t launch_stage(const StageArgs<T>& a, int block, hipStream_t s) {
  if (a.process == 0) return launch_adapt_tiles<T>(a, s);
  switch (columns_per_thread(a.g.nx, block)) {
    case 1: return launch_stage_ni<T, 1>(a, block, s);
    case 2: return launch_stage_ni<T, 2>(a, block, s);
    case 3: return launch_stage_ni<T, 3>(a, block, s);
    case 4: return launch_stage_ni<T, 4>(a, block, s);
    case 5: return launch_stage_ni<T, 5>(a, block, s);
    case 6: return launch_stage_ni<T, 6>(a, block, s);
    case 7: return launch_stage_ni<T, 7>(a, block, s);
    case 8: return launch_stage_ni<T, 8>(a, block, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_stage_batch(const StageArgs<T>* d_args, int nargs, int max_nz, const int2* d_titems, int ntitems,
                              const int2* d_items, int nitems, int grid, int block, int max_nx, size_t lds, int pipe,
                              hipStream_t s) {
  hipLaunchKernelGGL((k_capsum_batch<T>), dim3(max_nz, 2, nargs), dim3(64), 0, s, d_args, nargs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (columns_per_thread(max_nx, block)) {
    case 1: return launch_batch_ni<T, 1>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, pipe, s);
    case 2: return launch_batch_ni<T, 2>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, pipe, s);
    case 3: return launch_batch_ni<T, 3>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, pipe, s);
    case 4: return launch_batch_ni<T, 4>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, pipe, s);
    case 5: return launch_batch_ni<T, 5>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, pipe, s);
    case 6: return launch_batch_ni<T, 6>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, pipe, s);
    case 7: return launch_batch_ni<T, 7>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, pipe, s);
    case 8: return launch_batch_ni<T, 8>(d_args, d_titems, ntitems, d_items, nitems, grid, block, lds, pipe, s);
    default: return hipErrorInvalidValue;
  }
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
  template hipError_t launch_stage<T>(const StageArgs<T>&, int, hipStream_t);                                \
  template hipError_t launch_stage_batch<T>(const StageArgs<T>*, int, int, const int2*, int, const int2*, int,   \
                                            int, int, int, size_t, int, hipStream_t);                        \
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
