// Forward stage kernels of the leap-format dynamical core (gfx950).
//
// One workgroup owns one latitude row j: the scalar row j (Phi, p_s), the U
// row j and the V row j+1/2.  It walks the column top to bottom, level by
// level; each thread owns columns i = t, t+B, ... of the row and keeps its
// column sums in FP64 registers.  Rows that a leap difference reads at
// distance up to M (eq. 7, Table 6) are staged whole in LDS, so the periodic
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

// Deterministic FP64 row sum by wavefront 0: lane l adds i = l, l+64, ... in
// order, then a butterfly (commutative adds give every lane the same total).
__device__ __forceinline__ double wave_sum(double acc) {
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  return acc;
}

using C = double;

}  // namespace

// Largest workgroup per columns-per-thread: bounds the VGPR budget so that the FP64 column
// sums and one level's loads of every owned column stay in registers (768 threads: 170 VGPRs).
constexpr int max_block(int ni) { return ni <= 2 ? 768 : 512; }
int max_block_for(int nx, int block) { return block <= max_block(columns_per_thread(nx, block)) ? 1 : 0; }

namespace {

// ----------------------------------------------------------------------------------------------
// Adaptation: out = base + ch * A(in)
// ----------------------------------------------------------------------------------------------
// LDS: 2D rows P, l (rows j-1, j, j+1), q (rows j, j+1), leaped d+l and d+q on the U points of
// row j, and per level the leaped rows phi' and MU of row j.  Only the FP64 column sums live in
// registers across levels.
template <typename T, int NI>
__device__ void adapt_row(const StageArgs<T>& A, const int j, unsigned char* smem) {
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int B = blockDim.x, t = threadIdx.x;
  T* sPm = reinterpret_cast<T*>(smem);
  T* sP0 = sPm + nx;
  T* sP1 = sP0 + nx;
  T* sLm = sP1 + nx;
  T* sL0 = sLm + nx;
  T* sL1 = sL0 + nx;
  T* sQ0 = sL1 + nx;
  T* sQ1 = sQ0 + nx;
  T* sDl = sQ1 + nx;
  T* sDq = sDl + nx;
  T* sPhi = sDq + nx;
  T* sMU = sPhi + nx;
  double* sRed = reinterpret_cast<double*>(smem + ((12 * nx * sizeof(T) + 15) & ~size_t(15)));

  const bool isPole = (j == 0 || j == ny);
  const bool hasV = (j < ny);
  const int pidx = (j == 0) ? 0 : 1;
  const T p0 = (T)g.p0, b = (T)g.b, RT0 = (T)g.RT0;
  const C RT0c = g.RT0;
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
  auto UA = [&](int jr, int k, int i) -> T {
    if (jr == 0 || jr == ny) return T(0);
    return A.inU[(size_t)jr * row3 + (size_t)k * nx + i];
  };
  auto VA = [&](int jv, int k, int i) -> T { return A.inV[(size_t)jv * row3 + (size_t)k * nx + i]; };

  // ---- 2D rows
  for (int c = 0; c < NI; ++c) {
    const int i = t + c * B;
    if (i < nx) {
      const T ps0 = psA(j, i);
      sP0[i] = tsqrt<T>(ps0 / p0);
      sL0[i] = tlog<T>(ps0 / p0);
      sQ0[i] = sL0[i] + (T)g.phis[(size_t)j * nx + i] / RT0;
      if (j < ny) {
        const T ps1 = psA(j + 1, i);
        sP1[i] = tsqrt<T>(ps1 / p0);
        sL1[i] = tlog<T>(ps1 / p0);
        sQ1[i] = sL1[i] + (T)g.phis[(size_t)(j + 1) * nx + i] / RT0;
      }
      if (j > 0) {
        const T psm = psA(j - 1, i);
        sPm[i] = tsqrt<T>(psm / p0);
        sLm[i] = tlog<T>(psm / p0);
      }
    }
  }
  __syncthreads();
  const int Mj = isPole ? 1 : g.M[j];
  const int nj = (Mj + 1) / 2;
  const T dxj = isPole ? T(1) : (T)((double)Mj * g.a * g.s[j] * g.dlam);
  if (!isPole) {
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      if (i < nx) {
        sDl[i] = (sL0[wrp(i + nj, nx)] - sL0[wrp(i + 1 - nj, nx)]) / dxj;
        sDq[i] = (sQ0[wrp(i + nj, nx)] - sQ0[wrp(i + 1 - nj, nx)]) / dxj;
      }
    }
  }
  __syncthreads();

  C H0c[NI], H1c[NI], R0c[NI], R1c[NI], Sc[NI];
#pragma unroll
  for (int c = 0; c < NI; ++c) { H0c[c] = 0; H1c[c] = 0; R0c[c] = 0; R1c[c] = 0; Sc[c] = 0; }

  // ---- pass A: column totals H = sum_{l>=1} cl_l RT'_l (FP64) for phi' = H - R_k + cpk_k RT'_k
  if (hasV) {
    for (int k = 0; k < nz; ++k) {
      const C clk = g.cl[k];
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i < nx) {
          H0c[c] += clk * (C)(b * FA(j, k, i) / sP0[i]);
          H1c[c] += clk * (C)(b * FA(j + 1, k, i) / sP1[i]);
        }
      }
    }
  }

  // ---- pass B: top to bottom
  C Sp = 0;
  for (int k = 0; k < nz; ++k) {
    const C clk = g.cl[k], cpk = g.cpk[k];
    const C dsg = g.dsig[k], sgk = g.sig[k];
    // phase 1: every global load of this level, phi' and MU into LDS
    T Fj[NI], Fp[NI], RTj[NI], RTj1[NI], phij[NI], phij1[NI], Uj[NI], Ujm[NI], U1[NI], U1m[NI];
    T Vn[NI], Vnp[NI], Vs[NI], Vsp[NI], bF[NI], bU[NI], bV[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      Fj[c] = Fp[c] = RTj[c] = RTj1[c] = phij[c] = phij1[c] = Uj[c] = Ujm[c] = U1[c] = U1m[c] = T(0);
      Vn[c] = Vnp[c] = Vs[c] = Vsp[c] = bF[c] = bU[c] = bV[c] = T(0);
      if (i < nx) {
        const int ip1 = wrp(i + 1, nx), im1 = wrp(i - 1, nx);
        const size_t id = (size_t)j * row3 + (size_t)k * nx + i;
        Fj[c] = FA(j, k, i);
        RTj[c] = b * Fj[c] / sP0[i];
        if (hasV) {
          R0c[c] += clk * (C)RTj[c];
          phij[c] = (T)(H0c[c] - R0c[c] + cpk * (C)RTj[c]);
          RTj1[c] = b * FA(j + 1, k, i) / sP1[i];
          R1c[c] += clk * (C)RTj1[c];
          phij1[c] = (T)(H1c[c] - R1c[c] + cpk * (C)RTj1[c]);
          U1[c] = UA(j + 1, k, i);
          U1m[c] = UA(j + 1, k, im1);
          bV[c] = A.bV[id];
        }
        if (!isPole) {
          Fp[c] = FA(j, k, ip1);
          Uj[c] = UA(j, k, i);
          Ujm[c] = UA(j, k, im1);
          Vn[c] = VA(j, k, i);
          Vnp[c] = VA(j, k, ip1);
          Vs[c] = VA(j - 1, k, i);
          Vsp[c] = VA(j - 1, k, ip1);
          bF[c] = A.bF[id];
          bU[c] = A.bU[id];
          sPhi[i] = phij[c];
          sMU[i] = T(0.5) * (sP0[i] + sP0[ip1]) * Uj[c];
        }
      }
    }
    __syncthreads();

    if (!isPole) {
      const T dyS = (T)(g.a * g.s[j] * g.dth);
      const T dyA = (T)(g.a * g.dth);
      const T svj = (T)g.sv[j], svm = (T)g.sv[j - 1];
      const T fj = (T)g.f[j], cota = (T)(g.cot[j] / g.a);
      const T kap = (T)g.kappa;
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i >= nx) continue;
        const int ip1 = wrp(i + 1, nx), im1 = wrp(i - 1, nx);
        const size_t id = (size_t)j * row3 + (size_t)k * nx + i;
        const T PU = T(0.5) * (sP0[i] + sP0[ip1]);
        const T PUm = T(0.5) * (sP0[im1] + sP0[i]);
        const T PV0 = T(0.5) * (sP0[i] + sP1[i]);
        const T PVm = T(0.5) * (sPm[i] + sP0[i]);
        // divergence of the mass flux: leaped (x,x-1) -> (x+N-1, x-N) plus meridional
        const T D = (sMU[wrp(i + nj - 1, nx)] - sMU[wrp(i - nj, nx)]) / dxj +
                    (svj * (PV0 * Vn[c]) - svm * (PVm * Vs[c])) / dyS;
        const C Sk = Sc[c];
        Sc[c] += (C)D * dsg;
        // v . grad(l)
        const T u_i = Uj[c] / PU;
        const T u_m = Ujm[c] / PUm;
        const T zon = T(0.5) * (u_i * sDl[i] + u_m * sDl[im1]);
        const T mer = T(0.5) * ((Vn[c] / PV0) * (sL1[i] - sL0[i]) + (Vs[c] / PVm) * (sL0[i] - sLm[i])) / dyA;
        const C wp = ((C)zon + (C)mer) - (Sk + 0.5 * (C)D * dsg) / (sgk * (C)sP0[i] * (C)sP0[i]);
        const C TF = ((C)(b * sP0[i]) + (C)(kap * Fj[c])) * wp;
        A.oF[id] = (T)((C)bF[c] + A.ch * TF);
        // U at i+1/2: pressure gradient with leap (x+1,x) -> (x+N, x-N+1) and Coriolis
        const T dphi = (sPhi[wrp(i + nj, nx)] - sPhi[wrp(i + 1 - nj, nx)]) / dxj;
        const T RTp = b * Fp[c] / sP0[ip1];
        const T rtx = T(0.5) * (RTj[c] + RTp);
        const C pgf = (C)dphi + RT0c * (C)sDq[i] + (C)rtx * (C)sDl[i];
        const T VV = T(0.25) * (Vn[c] + Vnp[c] + Vs[c] + Vsp[c]);
        const T fs = fj + u_i * cota;
        const C TU = -(C)PU * pgf - (C)fs * (C)VV;
        A.oU[id] = (T)((C)bU[c] + A.ch * TU);
      }
    } else {
      // pole column: cap divergence and zonal-mean v.grad(l) from the adjacent V row
      const int jva = (j == 0) ? 0 : ny - 1;
      const T* sPa = (j == 0) ? sP1 : sPm;
      const T* sLa = (j == 0) ? sL1 : sLm;
      const T Pp = sP0[0];
      const T lp = sL0[0];
      if (t < 64) {
        C s1 = 0, s2 = 0;
        for (int i = t; i < nx; i += 64) {
          const T pv = T(0.5) * (Pp + sPa[i]);
          const T vv = VA(jva, k, i);
          s1 += (C)(pv * vv);
          s2 += (C)((vv / pv) * (j == 0 ? (sLa[i] - lp) : (lp - sLa[i])));
        }
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        if (t == 0) { sRed[0] = s1; sRed[1] = s2; }
      }
      __syncthreads();
      const C sgn = (j == 0) ? 1.0 : -1.0;
      const C Dp = sgn * g.a * g.dlam * g.sv[jva] * sRed[0] / g.acap;
      const C vglp = sRed[1] / ((double)nx * g.a * g.dth);
      const C Sk = Sp;
      Sp += Dp * dsg;
      const C wp = vglp - (Sk + 0.5 * Dp * dsg) / (sgk * (C)Pp * (C)Pp);
      const T Fpole = FA(j, k, 0);
      const C TF = ((C)(b * Pp) + (C)((T)g.kappa * Fpole)) * wp;
      const T val = (T)(A.pbase[pidx * (nz + 1) + k] + A.ch * TF);
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i < nx) {
          const size_t id = (size_t)j * row3 + (size_t)k * nx + i;
          A.oF[id] = val;
          A.oU[id] = T(0);
        }
      }
      if (t == 0) A.pout[pidx * (nz + 1) + k] = (double)val;
    }

    if (hasV) {
      const T dyA = (T)(g.a * g.dth);
      const T fvj = (T)g.fv[j], cotva = (T)(g.cotv[j] / g.a);
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i >= nx) continue;
        const int ip1 = wrp(i + 1, nx), im1 = wrp(i - 1, nx);
        const size_t idv = (size_t)j * row3 + (size_t)k * nx + i;
        const C pgf = ((C)(phij1[c] - phij[c]) + RT0c * (C)(sQ1[i] - sQ0[i]) +
                       (C)(T(0.5) * (RTj[c] + RTj1[c])) * (C)(sL1[i] - sL0[i])) / (C)dyA;
        const T u0i = Uj[c] / (T(0.5) * (sP0[i] + sP0[ip1]));
        const T u0m = Ujm[c] / (T(0.5) * (sP0[im1] + sP0[i]));
        const T u1i = U1[c] / (T(0.5) * (sP1[i] + sP1[ip1]));
        const T u1m = U1m[c] / (T(0.5) * (sP1[im1] + sP1[i]));
        const T UU = T(0.25) * (Ujm[c] + Uj[c] + U1m[c] + U1[c]);
        const T uu = T(0.25) * (u0m + u0i + u1m + u1i);
        const T fs = fvj + uu * cotva;
        const T PV0 = T(0.5) * (sP0[i] + sP1[i]);
        const C TV = -(C)PV0 * pgf + (C)fs * (C)UU;
        A.oV[idv] = (T)((C)bV[c] + A.ch * TV);
      }
    }
    __syncthreads();
  }

  // surface pressure: -p0 * Pi
  if (!isPole) {
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      if (i < nx) {
        const size_t id = (size_t)j * nx + i;
        A.oP[id] = (T)((C)A.bP[id] + A.ch * (-g.p0 * Sc[c]));
      }
    }
  } else {
    const T val = (T)(A.pbase[pidx * (nz + 1) + nz] + A.ch * (-g.p0 * Sp));
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      if (i < nx) A.oP[(size_t)j * nx + i] = val;
    }
    if (t == 0) A.pout[pidx * (nz + 1) + nz] = (double)val;
  }
}

// ----------------------------------------------------------------------------------------------
// Advection: out = base - ch * L(in), L in the IAP skew form, zonal part leaped
// ----------------------------------------------------------------------------------------------
// LDS: P rows j-1..j+2; per level the rows MU(j+1), Phi(j), U(j), V(j+1/2), u on the V row,
// v sin(theta) on V rows j-1/2 and j+1/2, and sigma-dot of row j at two half levels.
template <typename T, int NI>
__device__ void advect_row(const StageArgs<T>& A, const int j, unsigned char* smem) {
  const GeoDev& g = A.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int B = blockDim.x, t = threadIdx.x;
  T* sPm = reinterpret_cast<T*>(smem);    // P row j-1 (north pole WG: unused)
  T* sP0 = sPm + nx;                       // P row j
  T* sP1 = sP0 + nx;                       // P row j+1 (south pole WG: row ny-1)
  T* sP2 = sP1 + nx;                       // P row j+2
  T* sMU1 = sP2 + nx;                      // MU row j+1 at level k
  T* suv = sMU1 + nx;                      // u averaged to V row j+1/2
  T* sF = suv + nx;                        // Phi row j
  T* sU = sF + nx;                         // U row j
  T* sV = sU + nx;                         // V row j
  T* svtm = sV + nx;                       // v sin(theta) on V row j-1
  T* svt0 = svtm + nx;                     // v sin(theta) on V row j
  T* sSd = svt0 + nx;                      // sigma-dot row j at two half levels [2][nx]
  double* sRed = reinterpret_cast<double*>(smem + ((13 * nx * sizeof(T) + 15) & ~size_t(15)));

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
  auto UA = [&](int jr, int k, int i) -> T {
    if (jr <= 0 || jr >= ny) return T(0);
    return A.inU[(size_t)jr * row3 + (size_t)k * nx + i];
  };
  auto VA = [&](int jv, int k, int i) -> T { return A.inV[(size_t)jv * row3 + (size_t)k * nx + i]; };

  const int ja = (j == 0) ? 1 : ny - 1;   // row next to a pole
  for (int c = 0; c < NI; ++c) {
    const int i = t + c * B;
    if (i < nx) {
      sP0[i] = tsqrt<T>(psA(j, i) / p0);
      sP1[i] = tsqrt<T>(psA(hasV ? j + 1 : ja, i) / p0);
      if (j >= 1) sPm[i] = tsqrt<T>(psA(j - 1, i) / p0);
      if (j + 2 <= ny) sP2[i] = tsqrt<T>(psA(j + 2, i) / p0);
      sSd[i] = T(0);
      sSd[nx + i] = T(0);
    }
  }
  __syncthreads();

  const int Mj = isPole ? 1 : g.M[j], nj = (Mj + 1) / 2;
  const int Mj1 = j1Int ? g.M[j + 1] : 1, nj1 = (Mj1 + 1) / 2;
  const T dxj = isPole ? T(1) : (T)((double)Mj * g.a * g.s[j] * g.dlam);
  const T dxj1 = j1Int ? (T)((double)Mj1 * g.a * g.s[j + 1] * g.dlam) : T(1);
  const T dySj = isPole ? T(1) : (T)(g.a * g.s[j] * g.dth);
  const T dySj1 = j1Int ? (T)(g.a * g.s[j + 1] * g.dth) : T(1);
  auto PU0 = [&](int p) -> T { return T(0.5) * (sP0[p] + sP0[wrp(p + 1, nx)]); };
  auto PU1 = [&](int p) -> T { return T(0.5) * (sP1[p] + sP1[wrp(p + 1, nx)]); };

  C Pi0[NI], Pi1[NI], S0[NI], S1[NI], sd0c[NI], sd1c[NI];
#pragma unroll
  for (int c = 0; c < NI; ++c) { Pi0[c] = Pi1[c] = S0[c] = S1[c] = sd0c[c] = sd1c[c] = 0; }

  // divergence of rows j and j+1 at level k from the LDS rows sU (row j) and sMU1 (row j+1) and the
  // V values Vj (row j), Vm (row j-1), V1 (row j+1) of the own column.
  auto div_rows = [&](int k, const T* Vj, const T* Vm, const T* V1, C* D0, C* D1) {
    const bool needPole = isPole || (hasV && j1Pole);
    if (needPole) {
      if (t < 64) {
        C s = 0;
        const int jv = (j == 0) ? 0 : ny - 1;
        for (int i = t; i < nx; i += 64) {
          // the V row next to the pole with P of its two scalar rows: for j == 0 rows 0,1 (sP0,sP1);
          // j == ny: pole, ny-1 (sP0,sP1); j == ny-1: ny-1, pole (sP0,sP1)
          const T pv = T(0.5) * (sP0[i] + sP1[i]);
          s += (C)(pv * VA(jv, k, i));
        }
        s = wave_sum(s);
        if (t == 0) sRed[0] = s;
      }
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      D0[c] = 0; D1[c] = 0;
      if (i >= nx) continue;
      if (isPole) {
        const int jv = (j == 0) ? 0 : ny - 1;
        const C sgn = (j == 0) ? 1.0 : -1.0;
        D0[c] = sgn * g.a * g.dlam * g.sv[jv] * sRed[0] / g.acap;
      } else {
        const int pa = wrp(i + nj - 1, nx), pb = wrp(i - nj, nx);
        const T D = (PU0(pa) * sU[pa] - PU0(pb) * sU[pb]) / dxj +
                    ((T)g.sv[j] * (T(0.5) * (sP0[i] + sP1[i]) * Vj[c]) -
                     (T)g.sv[j - 1] * (T(0.5) * (sPm[i] + sP0[i]) * Vm[c])) / dySj;
        D0[c] = (C)D;
      }
      if (hasV) {
        if (j1Pole) {
          D1[c] = -g.a * g.dlam * g.sv[ny - 1] * sRed[0] / g.acap;
        } else {
          const T D = (sMU1[wrp(i + nj1 - 1, nx)] - sMU1[wrp(i - nj1, nx)]) / dxj1 +
                      ((T)g.sv[j + 1] * (T(0.5) * (sP1[i] + sP2[i]) * V1[c]) -
                       (T)g.sv[j] * (T(0.5) * (sP0[i] + sP1[i]) * Vj[c])) / dySj1;
          D1[c] = (C)D;
        }
      }
    }
  };

  // ---- pass A: column totals Pi for rows j and j+1
  for (int k = 0; k < nz; ++k) {
    T Vj[NI], Vm[NI], V1[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      Vj[c] = Vm[c] = V1[c] = T(0);
      if (i < nx) {
        sU[i] = UA(j, k, i);
        if (j1Int) sMU1[i] = PU1(i) * UA(j + 1, k, i);
        if (hasV) Vj[c] = VA(j, k, i);
        if (j >= 1) Vm[c] = VA(j - 1, k, i);
        if (j + 1 < ny) V1[c] = VA(j + 1, k, i);
      }
    }
    __syncthreads();
    C D0[NI], D1[NI];
    div_rows(k, Vj, Vm, V1, D0, D1);
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      Pi0[c] += D0[c] * g.dsig[k];
      Pi1[c] += D1[c] * g.dsig[k];
    }
    __syncthreads();
  }

  // ---- pass B
  const C cc = g.a * g.dlam / (2.0 * g.acap);
  for (int k = 0; k < nz; ++k) {
    const C dsg = g.dsig[k];
    const int par = k & 1, parn = (k + 1) & 1;
    // phase 1: loads of this level; LDS rows
    T Vj[NI], Vm[NI], V1[NI], Fn[NI], Fs[NI], Fup[NI], Fdn[NI], Un[NI], Us[NI], Uup[NI], Udn[NI];
    T Vup[NI], Vdn[NI], bF[NI], bU[NI], bV[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      Vj[c] = Vm[c] = V1[c] = Fn[c] = Fs[c] = Fup[c] = Fdn[c] = Un[c] = Us[c] = Uup[c] = Udn[c] = T(0);
      Vup[c] = Vdn[c] = bF[c] = bU[c] = bV[c] = T(0);
      if (i < nx) {
        const size_t id = (size_t)j * row3 + (size_t)k * nx + i;
        const T Fj = FA(j, k, i);
        const T Uj = UA(j, k, i);
        sF[i] = Fj;
        sU[i] = Uj;
        const T u0 = isPole ? T(0) : Uj / PU0(i);
        const T U1 = UA(j + 1, k, i);
        if (j1Int) sMU1[i] = PU1(i) * U1;
        if (hasV) {
          Vj[c] = VA(j, k, i);
          sV[i] = Vj[c];
          svt0[i] = Vj[c] / (T(0.5) * (sP0[i] + sP1[i])) * (T)g.sv[j];
          const T u1 = j1Int ? U1 / PU1(i) : T(0);
          suv[i] = T(0.5) * (u0 + u1);
          bV[c] = A.bV[id];
          if (k > 0) Vup[c] = VA(j, k - 1, i);
          if (k + 1 < nz) Vdn[c] = VA(j, k + 1, i);
        }
        if (j >= 1) {
          Vm[c] = VA(j - 1, k, i);
          svtm[i] = Vm[c] / (T(0.5) * (sPm[i] + sP0[i])) * (T)g.sv[j - 1];
        }
        if (j + 1 < ny) V1[c] = VA(j + 1, k, i);
        if (k > 0) Fup[c] = FA(j, k - 1, i);
        if (k + 1 < nz) Fdn[c] = FA(j, k + 1, i);
        if (!isPole) {
          Fn[c] = FA(j + 1, k, i);
          Fs[c] = FA(j - 1, k, i);
          Un[c] = U1;
          Us[c] = UA(j - 1, k, i);
          if (k > 0) Uup[c] = UA(j, k - 1, i);
          if (k + 1 < nz) Udn[c] = UA(j, k + 1, i);
          bF[c] = A.bF[id];
          bU[c] = A.bU[id];
        }
      }
    }
    __syncthreads();
    C D0[NI], D1[NI];
    div_rows(k, Vj, Vm, V1, D0, D1);
    C sd0n[NI], sd1n[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const int i = t + c * B;
      S0[c] += D0[c] * dsg;
      S1[c] += D1[c] * dsg;
      sd0n[c] = 0; sd1n[c] = 0;
      if (k + 1 < nz && i < nx) {
        const C sh = g.sigh[k + 1];
        sd0n[c] = (sh * Pi0[c] - S0[c]) / ((C)sP0[i] * (C)sP0[i]);
        if (hasV) sd1n[c] = (sh * Pi1[c] - S1[c]) / ((C)sP1[i] * (C)sP1[i]);
      }
      if (i < nx) sSd[parn * nx + i] = (T)sd0n[c];
    }
    // pole: meridional cap flux of Phi (needs every column of the adjacent rows)
    if (isPole) {
      if (t < 64) {
        C s = 0;
        const int jv = (j == 0) ? 0 : ny - 1;
        for (int i = t; i < nx; i += 64) {
          const T pv = T(0.5) * (sP0[i] + sP1[i]);
          const T vt = VA(jv, k, i) / pv * (T)g.sv[jv];
          s += (C)(vt * FA(ja, k, i));
        }
        s = wave_sum(s);
        if (t == 0) sRed[1] = s;
      }
    }
    __syncthreads();

    if (!isPole) {
      const T dx2 = T(2) * dxj;
      const T dy2 = T(2) * dySj;
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i >= nx) continue;
        const size_t id = (size_t)j * row3 + (size_t)k * nx + i;
        const int ip1 = wrp(i + 1, nx);
        auto u0 = [&](int p) -> T { return sU[p] / PU0(p); };
        // Phi: zonal (x+1,x-1) -> (x+2N-1, x-2N+1), u at the midpoints
        const int qa = wrp(i + nj - 1, nx), qb = wrp(i - nj, nx);
        const T L1 = (u0(qa) * sF[wrp(i + Mj, nx)] - u0(qb) * sF[wrp(i - Mj, nx)]) / dx2;
        const T L2 = (svt0[i] * Fn[c] - svtm[i] * Fs[c]) / dy2;
        C L3 = 0;
        if (k + 1 < nz) L3 += sd0n[c] * (C)Fdn[c];
        if (k > 0) L3 -= sd0c[c] * (C)Fup[c];
        L3 /= (2.0 * dsg);
        const C TF = -((C)L1 + (C)L2 + L3);
        A.oF[id] = (T)((C)bF[c] + A.ch * TF);
        // U: same leap on U points with u averaged to integer points
        const int pA = wrp(i + nj, nx), pB = wrp(i + 1 - nj, nx);
        const T ubA = T(0.5) * (u0(wrp(pA - 1, nx)) + u0(pA));
        const T ubB = T(0.5) * (u0(wrp(pB - 1, nx)) + u0(pB));
        const T U1v = (ubA * sU[wrp(i + Mj, nx)] - ubB * sU[wrp(i - Mj, nx)]) / dx2;
        const T vtn = T(0.5) * (svt0[i] + svt0[ip1]);
        const T vts = T(0.5) * (svtm[i] + svtm[ip1]);
        const T U2v = (vtn * Un[c] - vts * Us[c]) / dy2;
        C U3 = 0;
        if (k + 1 < nz) U3 += (C)(T(0.5) * (sSd[parn * nx + i] + sSd[parn * nx + ip1])) * (C)Udn[c];
        if (k > 0) U3 -= (C)(T(0.5) * (sSd[par * nx + i] + sSd[par * nx + ip1])) * (C)Uup[c];
        U3 /= (2.0 * dsg);
        const C TU = -((C)U1v + (C)U2v + U3);
        A.oU[id] = (T)((C)bU[c] + A.ch * TU);
      }
    } else {
      const C sgn = (j == 0) ? 1.0 : -1.0;
      const C L2 = sgn * cc * sRed[1];
      C L3 = 0;
      if (k + 1 < nz) L3 += sd0n[0] * (C)FA(j, k + 1, 0);
      if (k > 0) L3 -= sd0c[0] * (C)FA(j, k - 1, 0);
      L3 /= (2.0 * dsg);
      const C TF = -(L2 + L3);
      const T val = (T)(A.pbase[pidx * (nz + 1) + k] + A.ch * TF);
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i < nx) {
          const size_t id = (size_t)j * row3 + (size_t)k * nx + i;
          A.oF[id] = val;
          A.oU[id] = T(0);
        }
      }
      if (t == 0) A.pout[pidx * (nz + 1) + k] = (double)val;
    }

    if (hasV) {
      const int Mv = g.Mv[j], nv = (Mv + 1) / 2;
      const T dxv2 = (T)(2.0 * (double)Mv * g.a * g.sv[j] * g.dlam);
      const T dyv2 = (T)(2.0 * g.a * g.sv[j] * g.dth);
#pragma unroll
      for (int c = 0; c < NI; ++c) {
        const int i = t + c * B;
        if (i >= nx) continue;
        const size_t idv = (size_t)j * row3 + (size_t)k * nx + i;
        const T L1 = (suv[wrp(i + nv - 1, nx)] * sV[wrp(i + Mv, nx)] - suv[wrp(i - nv, nx)] * sV[wrp(i - Mv, nx)]) / dxv2;
        T L2 = T(0);
        if (j + 1 < ny) {
          const T vt1 = V1[c] / (T(0.5) * (sP1[i] + sP2[i])) * (T)g.sv[j + 1];
          L2 += T(0.5) * (svt0[i] + vt1) * V1[c];
        }
        if (j > 0) L2 -= T(0.5) * (svtm[i] + svt0[i]) * Vm[c];
        L2 = L2 / dyv2;
        C L3 = 0;
        if (k + 1 < nz) L3 += 0.5 * (sd0n[c] + sd1n[c]) * (C)Vdn[c];
        if (k > 0) L3 -= 0.5 * (sd0c[c] + sd1c[c]) * (C)Vup[c];
        L3 /= (2.0 * dsg);
        const C TV = -((C)L1 + (C)L2 + L3);
        A.oV[idv] = (T)((C)bV[c] + A.ch * TV);
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

// One launch per stage; the process is a template parameter so that the
// adaptation and advection kernels are separate symbols in a profile.
template <typename T, int NI, int PROC>
__global__ void __launch_bounds__(max_block(NI)) k_stage(StageArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int j = xcd_row(blockIdx.x, a.g.ny + 1);
  if (PROC == 0) adapt_row<T, NI>(a, j, smem);
  else advect_row<T, NI>(a, j, smem);
}

// Persistent batched stage: work item w = (member, row); block b takes items b, b+G, ...
template <typename T, int NI>
__global__ void __launch_bounds__(max_block(NI)) k_stage_batch(const StageArgs<T>* __restrict__ args,
                                                     const int2* __restrict__ items, int nitems) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    const int2 it = items[w];
    if (it.x < 0) continue;
    const StageArgs<T> a = args[it.x];
    if (a.process == 0) adapt_row<T, NI>(a, it.y, smem);
    else if (a.process == 1) advect_row<T, NI>(a, it.y, smem);
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
  if (a.process == 0) {
    e = allow_lds<k_stage<T, NI, 0>>(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stage<T, NI, 0>), dim3(a.g.ny + 1), dim3(block), lds, s, a);
  } else {
    e = allow_lds<k_stage<T, NI, 1>>(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stage<T, NI, 1>), dim3(a.g.ny + 1), dim3(block), lds, s, a);
  }
  return hipGetLastError();
}

template <typename T, int NI>
hipError_t launch_batch_ni(const StageArgs<T>* d_args, const int2* d_items, int nitems, int grid, int block,
                           int max_nx, hipStream_t s) {
  const size_t lds = std::max(stage_lds_bytes(0, max_nx, sizeof(T)), stage_lds_bytes(1, max_nx, sizeof(T)));
  hipError_t e = allow_lds<k_stage_batch<T, NI>>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_stage_batch<T, NI>), dim3(grid), dim3(block), lds, s, d_args, d_items, nitems);
  return hipGetLastError();
}

}  // namespace

size_t stage_lds_bytes(int process, int nx, int elem) {
  const size_t rows = (process == 0) ? 12 : 13;
  return ((rows * (size_t)nx * elem + 15) & ~size_t(15)) + 4 * sizeof(double);
}

int columns_per_thread(int nx, int block) { return (nx + block - 1) / block; }

template <typename T>
hipError_t launch_stage(const StageArgs<T>& a, int block, hipStream_t s) {
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
hipError_t launch_stage_batch(const StageArgs<T>* d_args, const int2* d_items, int nitems, int grid, int block,
                              int max_nx, hipStream_t s) {
  switch (columns_per_thread(max_nx, block)) {
    case 1: return launch_batch_ni<T, 1>(d_args, d_items, nitems, grid, block, max_nx, s);
    case 2: return launch_batch_ni<T, 2>(d_args, d_items, nitems, grid, block, max_nx, s);
    case 3: return launch_batch_ni<T, 3>(d_args, d_items, nitems, grid, block, max_nx, s);
    case 4: return launch_batch_ni<T, 4>(d_args, d_items, nitems, grid, block, max_nx, s);
    case 5: return launch_batch_ni<T, 5>(d_args, d_items, nitems, grid, block, max_nx, s);
    case 6: return launch_batch_ni<T, 6>(d_args, d_items, nitems, grid, block, max_nx, s);
    case 7: return launch_batch_ni<T, 7>(d_args, d_items, nitems, grid, block, max_nx, s);
    case 8: return launch_batch_ni<T, 8>(d_args, d_items, nitems, grid, block, max_nx, s);
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
                       int npartial, hipStream_t s) {
  (void)npartial;
  hipLaunchKernelGGL((k_diag<T>), dim3(g.ny + 1), dim3(256), 0, s, g, U, V, F, ps, partial);
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
  template hipError_t launch_stage_batch<T>(const StageArgs<T>*, const int2*, int, int, int, int, hipStream_t); \
  template hipError_t launch_pole_prep<T>(const GeoDev&, const T*, const T*, double*, hipStream_t);          \
  template hipError_t launch_diag<T>(const GeoDev&, const T*, const T*, const T*, const T*, double*, int,    \
                                     hipStream_t);                                                           \
  template hipError_t launch_nonfinite<T>(const T*, size_t, unsigned long long*, hipStream_t);               \
  template hipError_t launch_axpy_fill<T>(T*, const T*, size_t, hipStream_t);                                \
  template hipError_t launch_zero<T>(T*, size_t, hipStream_t);
DYC_INST(float)
DYC_INST(double)
template hipError_t launch_zero<unsigned long long>(unsigned long long*, size_t, hipStream_t);

}  // namespace dyc
