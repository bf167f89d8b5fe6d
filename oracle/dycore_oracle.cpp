// Plain FP64 CPU oracle of the leap-format dynamical-core step.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no code, header or table with the HIP path.
//
// What it computes (AGCM-3DLF, arXiv 2103.10114):
//   * eq. 1  : the IAP-transformed primitive equations for U, V, Phi, p_s
//   * eq. 2  : the split dF/dt = -L_F + A_F into advection and adaptation
//   * Sec. III-B, C grid: U at (x+1/2,y), V at (x,y+1/2), scalars at (x,y)
//   * eq. 5/6: central zonal difference and its leap-format generalisation
//   * eq. 7  : N_leap from the 45-degree reference spacing
//   * Table VII: the leap patterns (x+1,x)->(x+N,x-N+1), (x,x-1)->(x+N-1,x-N),
//              (x+1,x-1)->(x+2N-1,x-2N+1) with N the half width
//   * Alg. 1/2: the column sum and prefix sum behind the sigma-dot diagnosis
//     (one plain sequential scan per column; the blocked form of Alg. 2 is the
//     same sum regrouped)
//   * Sec. III-D (message aggregation): 3M adaptation and 3 advection calls
//     per step
// Every difference form that the paper names without printing it is a stated
// reading (R1..R24 in the design notes); the code follows those readings
// literally, in plain loops, in the paper's notation where one exists.
//
// The forward map is templated on the scalar type so that instantiating it
// with std::complex<double> gives the exact tangent-linear by complex step
// (Im f(x + i h dx) / h), an independent check on the hand-written adjoint.

#include <cmath>
#include <complex>
#include <cstring>
#include <cstdlib>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

using cplx = std::complex<double>;

namespace {

struct Geo {
  int nx, ny, nz;
  double a, omega, g, rd, cp, p0, t0, kappa, b;
  double dlam, dth, acap;
  std::vector<double> s, cot, f;        // scalar/U rows j = 0..ny (theta_j = j*dth)
  std::vector<double> sv, cotv, fv;     // V rows jv = 0..ny-1 (theta = (jv+1/2)*dth)
  std::vector<double> r, rv;            // eq. 7 ratio per row
  std::vector<int> M, n, Mv, nv;        // leap span (odd) and half width
  std::vector<double> sigh, sig, dsig, cl, cpk;
  std::vector<double> phis;             // (ny+1)*nx, pole rows replaced by their mean
  int filters = 0;                      // low-latitude filters after each outer step (Table IV rows 1-2)
  double kstar = 0.0;                   // p_s diffusion coefficient kappa* of eq. 1 (m^2/s)
};

// eq. 7 with res = dlam and cos(90deg - theta) = sin(theta); the result is
// rounded up, made odd (a U-point difference must land on U points), and kept
// below nx/2 so that i+M and i-M are distinct columns.
int leap_span(double sin_theta, double dlam, int nx, double* ratio) {
  const double num = std::asin(std::cos(M_PI / 4.0) * std::sin(dlam));
  const double den = std::asin(sin_theta * std::sin(dlam));
  const double r = num / den;
  *ratio = r;
  int M = (int)std::ceil(r - 1e-9);
  if (M < 1) M = 1;
  if (M % 2 == 0) M += 1;
  int cap = (nx - 1) / 2;
  if (cap % 2 == 0) cap -= 1;
  if (cap < 1) cap = 1;
  if (M > cap) M = cap;
  return M;
}

inline int wrap(int i, int nx) { int r = i % nx; return r < 0 ? r + nx : r; }

template <typename T> inline T tsqrt(T x) { return std::sqrt(x); }
template <typename T> inline T tlog(T x) { return std::log(x); }

// ---------------------------------------------------------------- state
template <typename T>
struct St {
  std::vector<T> U, V, F, ps;  // F is Phi
};

template <typename T>
struct Work {
  std::vector<T> pse, Fe, Ue;            // pole-read fields (pole rows = row means), U with pole rows 0
  std::vector<T> P, l, q;                // 2D scalar rows
  std::vector<T> RT, phi;                // 3D scalar: R T' = b Phi / P, hydrostatic deviation
  std::vector<T> PU, PV;                 // 2D at U rows / V rows
  std::vector<T> u, v, MU, MV;           // 3D at U / V points
  std::vector<T> D;                      // 3D scalar divergence of (MU, MV)
  std::vector<T> S;                      // (ny+1)*(nz+1)*nx prefix sums at half levels; S[nz] = Pi
  std::vector<T> sd;                     // (ny+1)*(nz+1)*nx sigma-dot at half levels
  std::vector<T> vgl, wp;                // 3D scalar: v.grad(l), omega/p
};

struct Sizes {
  int nx, ny, nz;
  size_t n2, n3, nv3, nh3;
  explicit Sizes(const Geo& g) : nx(g.nx), ny(g.ny), nz(g.nz) {
    n2 = (size_t)(ny + 1) * nx;
    n3 = (size_t)(ny + 1) * nz * nx;
    nv3 = (size_t)ny * nz * nx;
    nh3 = (size_t)(ny + 1) * (nz + 1) * nx;
  }
  size_t i3(int j, int k, int i) const { return ((size_t)j * nz + k) * nx + wrap(i, nx); }
  size_t i2(int j, int i) const { return (size_t)j * nx + wrap(i, nx); }
  size_t ih(int j, int h, int i) const { return ((size_t)j * (nz + 1) + h) * nx + wrap(i, nx); }
};

// ---------------------------------------------------------------- diagnosis (column diagnostics)
template <typename T>
void diagnose(const Geo& g, const St<T>& y, Work<T>& w) {
  const Sizes z(g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double a = g.a;
  w.pse.assign(z.n2, T(0)); w.Fe.assign(z.n3, T(0)); w.Ue.assign(z.n3, T(0));
  w.P.assign(z.n2, T(0)); w.l.assign(z.n2, T(0)); w.q.assign(z.n2, T(0));
  w.RT.assign(z.n3, T(0)); w.phi.assign(z.n3, T(0));
  w.PU.assign(z.n2, T(0)); w.PV.assign((size_t)ny * nx, T(0));
  w.u.assign(z.n3, T(0)); w.MU.assign(z.n3, T(0));
  w.v.assign(z.nv3, T(0)); w.MV.assign(z.nv3, T(0));
  w.D.assign(z.n3, T(0)); w.S.assign(z.nh3, T(0)); w.sd.assign(z.nh3, T(0));
  w.vgl.assign(z.n3, T(0)); w.wp.assign(z.n3, T(0));

  // Pole reads: a pole value is the mean of its stored (replicated) row.
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i) w.pse[z.i2(j, i)] = y.ps[z.i2(j, i)];
  for (int p : {0, ny}) {
    T m(0);
    for (int i = 0; i < nx; ++i) m += y.ps[z.i2(p, i)];
    m /= double(nx);
    for (int i = 0; i < nx; ++i) w.pse[z.i2(p, i)] = m;
  }
  w.Fe = y.F;
  for (int p : {0, ny})
    for (int k = 0; k < nz; ++k) {
      T m(0);
      for (int i = 0; i < nx; ++i) m += y.F[z.i3(p, k, i)];
      m /= double(nx);
      for (int i = 0; i < nx; ++i) w.Fe[z.i3(p, k, i)] = m;
    }
  w.Ue = y.U;
  for (int p : {0, ny})
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) w.Ue[z.i3(p, k, i)] = T(0);

  // IAP transform quantities on scalar rows: P = sqrt(ps/p0), l = ln(ps/p0), q = l + phis/(R T0)
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const T pr = w.pse[z.i2(j, i)] / g.p0;
      w.P[z.i2(j, i)] = tsqrt(pr);
      w.l[z.i2(j, i)] = tlog(pr);
      w.q[z.i2(j, i)] = w.l[z.i2(j, i)] + g.phis[z.i2(j, i)] / (g.rd * g.t0);
    }

  // R T' = b Phi / P
#pragma omp parallel for
  for (int j = 0; j <= ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) w.RT[z.i3(j, k, i)] = g.b * w.Fe[z.i3(j, k, i)] / w.P[z.i2(j, i)];

  // Hydrostatic deviation geopotential, zero at the surface (sigma = 1)
#pragma omp parallel for
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int k = 0; k < nz; ++k) {
        T acc = g.cpk[k] * w.RT[z.i3(j, k, i)];
        for (int l2 = k + 1; l2 < nz; ++l2) acc += g.cl[l2] * w.RT[z.i3(j, l2, i)];
        w.phi[z.i3(j, k, i)] = acc;
      }

  // Staggered P: PU at (i+1/2, j), PV at (i, j+1/2)
  for (int j = 1; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      w.PU[z.i2(j, i)] = 0.5 * (w.P[z.i2(j, i)] + w.P[z.i2(j, i + 1)]);
  for (int jv = 0; jv < ny; ++jv)
    for (int i = 0; i < nx; ++i)
      w.PV[z.i2(jv, i)] = 0.5 * (w.P[z.i2(jv, i)] + w.P[z.i2(jv + 1, i)]);

  // Velocities and mass fluxes
#pragma omp parallel for
  for (int j = 1; j < ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const size_t id = z.i3(j, k, i);
        w.u[id] = w.Ue[id] / w.PU[z.i2(j, i)];
        w.MU[id] = w.PU[z.i2(j, i)] * w.Ue[id];
      }
#pragma omp parallel for
  for (int jv = 0; jv < ny; ++jv)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const size_t id = z.i3(jv, k, i);
        w.v[id] = y.V[id] / w.PV[z.i2(jv, i)];
        w.MV[id] = w.PV[z.i2(jv, i)] * y.V[id];
      }

  // Divergence D of the mass flux: leaped zonal part (Table VII pattern (x,x-1) ->
  // (x+N-1, x-N)) plus the plain meridional part; cap divergences at the poles.
#pragma omp parallel for
  for (int j = 1; j < ny; ++j) {
    const int M = g.M[j], n = g.n[j];
    const double dx = M * a * g.s[j] * g.dlam;
    const double dy = a * g.s[j] * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const T zon = (w.MU[z.i3(j, k, i + n - 1)] - w.MU[z.i3(j, k, i - n)]) / dx;
        const T mer = (g.sv[j] * w.MV[z.i3(j, k, i)] - g.sv[j - 1] * w.MV[z.i3(j - 1, k, i)]) / dy;
        w.D[z.i3(j, k, i)] = zon + mer;
      }
  }
  for (int k = 0; k < nz; ++k) {
    T sn(0), ss(0);
    for (int i = 0; i < nx; ++i) {
      sn += w.MV[z.i3(0, k, i)];
      ss += w.MV[z.i3(ny - 1, k, i)];
    }
    const T dn = a * g.dlam * g.sv[0] * sn / g.acap;
    const T ds = -a * g.dlam * g.sv[ny - 1] * ss / g.acap;
    for (int i = 0; i < nx; ++i) {
      w.D[z.i3(0, k, i)] = dn;
      w.D[z.i3(ny, k, i)] = ds;
    }
  }

  // Column prefix sums S_h = sum_{k<h} D_k dsig_k (Alg. 1/2), Pi = S_nz
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i) {
      T acc(0);
      w.S[z.ih(j, 0, i)] = acc;
      for (int k = 0; k < nz; ++k) {
        acc = acc + w.D[z.i3(j, k, i)] * g.dsig[k];
        w.S[z.ih(j, k + 1, i)] = acc;
      }
    }

  // sigma-dot at half levels: P^2 sd_h = sigh_h Pi - S_h (zero at top and surface)
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const T P2 = w.P[z.i2(j, i)] * w.P[z.i2(j, i)];
      const T Pi = w.S[z.ih(j, nz, i)];
      for (int h = 1; h < nz; ++h)
        w.sd[z.ih(j, h, i)] = (g.sigh[h] * Pi - w.S[z.ih(j, h, i)]) / P2;
    }

  // v . grad(l) at scalar points
#pragma omp parallel for
  for (int j = 1; j < ny; ++j) {
    const int M = g.M[j], n = g.n[j];
    const double dx = M * a * g.s[j] * g.dlam;
    const double dy = a * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const T dl_r = (w.l[z.i2(j, i + n)] - w.l[z.i2(j, i + 1 - n)]) / dx;      // at i+1/2
        const T dl_l = (w.l[z.i2(j, i - 1 + n)] - w.l[z.i2(j, i - n)]) / dx;      // at i-1/2
        const T zon = 0.5 * (w.u[z.i3(j, k, i)] * dl_r + w.u[z.i3(j, k, i - 1)] * dl_l);
        const T mer = 0.5 * (w.v[z.i3(j, k, i)] * (w.l[z.i2(j + 1, i)] - w.l[z.i2(j, i)]) +
                             w.v[z.i3(j - 1, k, i)] * (w.l[z.i2(j, i)] - w.l[z.i2(j - 1, i)])) / dy;
        w.vgl[z.i3(j, k, i)] = zon + mer;
      }
  }
  for (int k = 0; k < nz; ++k) {
    T sn(0), ss(0);
    for (int i = 0; i < nx; ++i) {
      sn += w.v[z.i3(0, k, i)] * (w.l[z.i2(1, i)] - w.l[z.i2(0, i)]);
      ss += w.v[z.i3(ny - 1, k, i)] * (w.l[z.i2(ny, i)] - w.l[z.i2(ny - 1, i)]);
    }
    sn = sn / (double(nx) * a * g.dth);
    ss = ss / (double(nx) * a * g.dth);
    for (int i = 0; i < nx; ++i) {
      w.vgl[z.i3(0, k, i)] = sn;
      w.vgl[z.i3(ny, k, i)] = ss;
    }
  }

  // omega/p = v.grad(l) - (S_k + D_k dsig_k / 2) / (sig_k P^2)
  for (int j = 0; j <= ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const T P2 = w.P[z.i2(j, i)] * w.P[z.i2(j, i)];
        const T Sk = w.S[z.ih(j, k, i)] + 0.5 * w.D[z.i3(j, k, i)] * g.dsig[k];
        w.wp[z.i3(j, k, i)] = w.vgl[z.i3(j, k, i)] - Sk / (g.sig[k] * P2);
      }
}

// ---------------------------------------------------------------- adaptation tendency A
template <typename T>
void tend_A(const Geo& g, const St<T>& y, const Work<T>& w, St<T>& t) {
  const Sizes z(g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double a = g.a, RT0 = g.rd * g.t0;
  t.U.assign(z.n3, T(0)); t.V.assign(z.nv3, T(0)); t.F.assign(z.n3, T(0)); t.ps.assign(z.n2, T(0));

  // Phi: (b + kappa Phi / P) * Omega~, Omega~ = P * omega/p  ==  (b P + kappa Phi) * omega/p
  for (int j = 0; j <= ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const size_t id = z.i3(j, k, i);
        t.F[id] = (g.b * w.P[z.i2(j, i)] + g.kappa * w.Fe[id]) * w.wp[id];
      }
  // p_s: -p0 * Pi
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i) t.ps[z.i2(j, i)] = -g.p0 * w.S[z.ih(j, nz, i)];
  // p_s diffusion kappa* D_sa (eq. 1, p_s line): the horizontal Laplacian of p_s in flux form on
  // the C grid, zonally the leaped difference of the leaped difference, (F_{i+M} - 2 F_i + F_{i-M})
  // / (M dx)^2; meridionally the divergence of the face gradients; at a pole the outward gradient
  // flux through the cap edge over the cap area
  if (g.kstar != 0.0) {
    for (int j = 1; j < ny; ++j) {
      const int M = g.M[j];
      const double dx = M * a * g.s[j] * g.dlam;
      const double dy2 = a * a * g.s[j] * g.dth * g.dth;
      for (int i = 0; i < nx; ++i) {
        const T zon = (w.pse[z.i2(j, i + M)] - 2.0 * w.pse[z.i2(j, i)] + w.pse[z.i2(j, i - M)]) / (dx * dx);
        const T mer = (g.sv[j] * (w.pse[z.i2(j + 1, i)] - w.pse[z.i2(j, i)]) -
                       g.sv[j - 1] * (w.pse[z.i2(j, i)] - w.pse[z.i2(j - 1, i)])) / dy2;
        t.ps[z.i2(j, i)] += g.kstar * (zon + mer);
      }
    }
    T fn(0), fs(0);
    for (int i = 0; i < nx; ++i) {
      fn += w.pse[z.i2(1, i)] - w.pse[z.i2(0, i)];
      fs += w.pse[z.i2(ny - 1, i)] - w.pse[z.i2(ny, i)];
    }
    const T dn = g.sv[0] * g.dlam / (g.acap * g.dth) * fn;
    const T ds = g.sv[ny - 1] * g.dlam / (g.acap * g.dth) * fs;
    for (int i = 0; i < nx; ++i) {
      t.ps[z.i2(0, i)] += g.kstar * dn;
      t.ps[z.i2(ny, i)] += g.kstar * ds;
    }
  }

  // U: -P^U [d+ phi' + R T0 d+ q + <RT'>^x d+ l] - f* <<V>>, leap pattern (x+1,x) -> (x+N, x-N+1)
#pragma omp parallel for
  for (int j = 1; j < ny; ++j) {
    const int M = g.M[j], n = g.n[j];
    const double dx = M * a * g.s[j] * g.dlam;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const T dphi = (w.phi[z.i3(j, k, i + n)] - w.phi[z.i3(j, k, i + 1 - n)]) / dx;
        const T dq = (w.q[z.i2(j, i + n)] - w.q[z.i2(j, i + 1 - n)]) / dx;
        const T dl = (w.l[z.i2(j, i + n)] - w.l[z.i2(j, i + 1 - n)]) / dx;
        const T rtx = 0.5 * (w.RT[z.i3(j, k, i)] + w.RT[z.i3(j, k, i + 1)]);
        const T pgf = dphi + RT0 * dq + rtx * dl;
        const T VV = 0.25 * (y.V[z.i3(j, k, i)] + y.V[z.i3(j, k, i + 1)] +
                             y.V[z.i3(j - 1, k, i)] + y.V[z.i3(j - 1, k, i + 1)]);
        const T fs = g.f[j] + w.u[z.i3(j, k, i)] * g.cot[j] / a;
        t.U[z.i3(j, k, i)] = -w.PU[z.i2(j, i)] * pgf - fs * VV;
      }
  }
  // V: -P^V [dy phi' + R T0 dy q + <RT'>^y dy l] + f* <<U>>
#pragma omp parallel for
  for (int jv = 0; jv < ny; ++jv) {
    const double dy = a * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const T dphi = w.phi[z.i3(jv + 1, k, i)] - w.phi[z.i3(jv, k, i)];
        const T dq = w.q[z.i2(jv + 1, i)] - w.q[z.i2(jv, i)];
        const T dl = w.l[z.i2(jv + 1, i)] - w.l[z.i2(jv, i)];
        const T rty = 0.5 * (w.RT[z.i3(jv, k, i)] + w.RT[z.i3(jv + 1, k, i)]);
        const T pgf = (dphi + RT0 * dq + rty * dl) / dy;
        const T UU = 0.25 * (w.Ue[z.i3(jv, k, i - 1)] + w.Ue[z.i3(jv, k, i)] +
                             w.Ue[z.i3(jv + 1, k, i - 1)] + w.Ue[z.i3(jv + 1, k, i)]);
        const T uu = 0.25 * (w.u[z.i3(jv, k, i - 1)] + w.u[z.i3(jv, k, i)] +
                             w.u[z.i3(jv + 1, k, i - 1)] + w.u[z.i3(jv + 1, k, i)]);
        const T fs = g.fv[jv] + uu * g.cotv[jv] / a;
        t.V[z.i3(jv, k, i)] = -w.PV[z.i2(jv, i)] * pgf + fs * UU;
      }
  }
}

// ---------------------------------------------------------------- advection tendency -L
template <typename T>
void tend_L(const Geo& g, const St<T>& y, const Work<T>& w, St<T>& t) {
  const Sizes z(g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double a = g.a;
  t.U.assign(z.n3, T(0)); t.V.assign(z.nv3, T(0)); t.F.assign(z.n3, T(0)); t.ps.assign(z.n2, T(0));
  auto vt = [&](int jv, int k, int i) -> T { return w.v[z.i3(jv, k, i)] * g.sv[jv]; };

  // Phi at interior scalar rows: zonal (x+1,x-1) -> (x+2N-1, x-2N+1) with the advecting
  // u at the midpoints (Table VII "Ustar" positions), plain meridional and vertical parts.
#pragma omp parallel for
  for (int j = 1; j < ny; ++j) {
    const int M = g.M[j], n = g.n[j];
    const double dx2 = 2.0 * M * a * g.s[j] * g.dlam;
    const double dy2 = 2.0 * a * g.s[j] * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const T L1 = (w.u[z.i3(j, k, i + n - 1)] * w.Fe[z.i3(j, k, i + M)] -
                      w.u[z.i3(j, k, i - n)] * w.Fe[z.i3(j, k, i - M)]) / dx2;
        const T L2 = (vt(j, k, i) * w.Fe[z.i3(j + 1, k, i)] - vt(j - 1, k, i) * w.Fe[z.i3(j - 1, k, i)]) / dy2;
        T L3(0);
        if (k + 1 < nz) L3 += w.sd[z.ih(j, k + 1, i)] * w.Fe[z.i3(j, k + 1, i)];
        if (k > 0) L3 -= w.sd[z.ih(j, k, i)] * w.Fe[z.i3(j, k - 1, i)];
        L3 = L3 / (2.0 * g.dsig[k]);
        t.F[z.i3(j, k, i)] = -(L1 + L2 + L3);
      }
  }
  // Phi at the poles: cap flux form of the meridional part, vertical part per pole column
  const double cc = a * g.dlam / (2.0 * g.acap);
  for (int k = 0; k < nz; ++k) {
    T sn(0), ss(0);
    for (int i = 0; i < nx; ++i) {
      sn += vt(0, k, i) * w.Fe[z.i3(1, k, i)];
      ss += vt(ny - 1, k, i) * w.Fe[z.i3(ny - 1, k, i)];
    }
    const T L2n = cc * sn, L2s = -cc * ss;
    for (int p : {0, ny}) {
      const T L2 = (p == 0) ? L2n : L2s;
      for (int i = 0; i < nx; ++i) {
        T L3(0);
        if (k + 1 < nz) L3 += w.sd[z.ih(p, k + 1, i)] * w.Fe[z.i3(p, k + 1, i)];
        if (k > 0) L3 -= w.sd[z.ih(p, k, i)] * w.Fe[z.i3(p, k - 1, i)];
        L3 = L3 / (2.0 * g.dsig[k]);
        t.F[z.i3(p, k, i)] = -(L2 + L3);
      }
    }
  }

  // U at interior rows: zonal (x+1,x-1) -> (x+2N-1,x-2N+1) on U points with the advecting
  // u averaged to the integer midpoints (Table VII "Ustar" (x+1,x) -> (x+N, x-N+1)).
#pragma omp parallel for
  for (int j = 1; j < ny; ++j) {
    const int M = g.M[j], n = g.n[j];
    const double dx2 = 2.0 * M * a * g.s[j] * g.dlam;
    const double dy2 = 2.0 * a * g.s[j] * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        auto ub = [&](int p) -> T { return 0.5 * (w.u[z.i3(j, k, p - 1)] + w.u[z.i3(j, k, p)]); };
        const T L1 = (ub(i + n) * w.Ue[z.i3(j, k, i + M)] - ub(i + 1 - n) * w.Ue[z.i3(j, k, i - M)]) / dx2;
        auto vtu = [&](int jv) -> T { return 0.5 * (vt(jv, k, i) + vt(jv, k, i + 1)); };
        const T L2 = (vtu(j) * w.Ue[z.i3(j + 1, k, i)] - vtu(j - 1) * w.Ue[z.i3(j - 1, k, i)]) / dy2;
        auto sdu = [&](int h) -> T { return 0.5 * (w.sd[z.ih(j, h, i)] + w.sd[z.ih(j, h, i + 1)]); };
        T L3(0);
        if (k + 1 < nz) L3 += sdu(k + 1) * w.Ue[z.i3(j, k + 1, i)];
        if (k > 0) L3 -= sdu(k) * w.Ue[z.i3(j, k - 1, i)];
        L3 = L3 / (2.0 * g.dsig[k]);
        t.U[z.i3(j, k, i)] = -(L1 + L2 + L3);
      }
  }

  // V rows: zonal leap with the V row's own span and u averaged meridionally to (i+1/2, j+1/2)
#pragma omp parallel for
  for (int jv = 0; jv < ny; ++jv) {
    const int M = g.Mv[jv], n = g.nv[jv];
    const double dx2 = 2.0 * M * a * g.sv[jv] * g.dlam;
    const double dy2 = 2.0 * a * g.sv[jv] * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        auto uv = [&](int p) -> T { return 0.5 * (w.u[z.i3(jv, k, p)] + w.u[z.i3(jv + 1, k, p)]); };
        const T L1 = (uv(i + n - 1) * y.V[z.i3(jv, k, i + M)] - uv(i - n) * y.V[z.i3(jv, k, i - M)]) / dx2;
        // meridional velocity at scalar rows, zero on the pole rows
        auto vts = [&](int js) -> T {
          if (js <= 0 || js >= ny) return T(0);
          return 0.5 * (vt(js - 1, k, i) + vt(js, k, i));
        };
        T L2(0);
        if (jv + 1 < ny) L2 += vts(jv + 1) * y.V[z.i3(jv + 1, k, i)];
        if (jv > 0) L2 -= vts(jv) * y.V[z.i3(jv - 1, k, i)];
        L2 = L2 / dy2;
        auto sdv = [&](int h) -> T { return 0.5 * (w.sd[z.ih(jv, h, i)] + w.sd[z.ih(jv + 1, h, i)]); };
        T L3(0);
        if (k + 1 < nz) L3 += sdv(k + 1) * y.V[z.i3(jv, k + 1, i)];
        if (k > 0) L3 -= sdv(k) * y.V[z.i3(jv, k - 1, i)];
        L3 = L3 / (2.0 * g.dsig[k]);
        t.V[z.i3(jv, k, i)] = -(L1 + L2 + L3);
      }
  }
}

// ---------------------------------------------------------------- stage / RK3 / step
template <typename T>
void tendency(const Geo& g, const St<T>& y, int which, St<T>& t) {
  Work<T> w;
  diagnose(g, y, w);
  if (which == 0) tend_A(g, y, w, t); else tend_L(g, y, w, t);
}

// out = base + ch * T(yin); pole rows: mean of the base row + ch * pole tendency, replicated;
// U pole rows are zero.
template <typename T>
void stage(const Geo& g, const St<T>& base, const St<T>& yin, double ch, int which, St<T>& out) {
  const Sizes z(g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  St<T> t;
  tendency(g, yin, which, t);
  out.U.assign(z.n3, T(0)); out.V.assign(z.nv3, T(0)); out.F.assign(z.n3, T(0)); out.ps.assign(z.n2, T(0));
  for (int j = 1; j < ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const size_t id = z.i3(j, k, i);
        out.U[id] = base.U[id] + ch * t.U[id];
        out.F[id] = base.F[id] + ch * t.F[id];
      }
  for (size_t id = 0; id < z.nv3; ++id) out.V[id] = base.V[id] + ch * t.V[id];
  for (int j = 1; j < ny; ++j)
    for (int i = 0; i < nx; ++i) out.ps[z.i2(j, i)] = base.ps[z.i2(j, i)] + ch * t.ps[z.i2(j, i)];
  for (int p : {0, ny}) {
    T m(0);
    for (int i = 0; i < nx; ++i) m += base.ps[z.i2(p, i)];
    m /= double(nx);
    for (int i = 0; i < nx; ++i) out.ps[z.i2(p, i)] = m + ch * t.ps[z.i2(p, i)];
    for (int k = 0; k < nz; ++k) {
      T mf(0);
      for (int i = 0; i < nx; ++i) mf += base.F[z.i3(p, k, i)];
      mf /= double(nx);
      for (int i = 0; i < nx; ++i) out.F[z.i3(p, k, i)] = mf + ch * t.F[z.i3(p, k, i)];
    }
  }
}

// Wicker-Skamarock RK3: y1 = y + h/3 T(y), y2 = y + h/2 T(y1), y+ = y + h T(y2)
template <typename T>
void rk3(const Geo& g, St<T>& y, double h, int which) {
  St<T> y1, y2, y3;
  stage(g, y, y, h / 3.0, which, y1);
  stage(g, y, y1, h / 2.0, which, y2);
  stage(g, y, y2, h, which, y3);
  y = y3;
}

// ---------------------------------------------------------------- low-latitude filters
// The filters the leap format keeps equatorward of 70 degrees (Sec. III-B, Table IV rows 1-2),
// one zonal row at a time, in the readings of the design notes:
//   |lat| < 38 deg:        the simplified filter removes the 2-dlam wave, F_x -= (-1)^x A with
//                          A = (1/I) sum_x' (-1)^x' F_x' (x from 0, I = nx even);
//   38 <= |lat| <= 70 deg: the 3-point operator F_x + r (F_{x-1} - 2 F_x + F_{x+1}), with
//                          r = (1 - cos(lat) / cos 38deg) / 4, so that the 2-dlam wave keeps the
//                          fraction cos(lat) / cos 38deg of its amplitude (the ratio of the row's
//                          zonal spacing to the spacing at 38 degrees);
//   |lat| > 70 deg:        no filter (the leap takes its place).
// The latitude of a row is 90 (ny - 2j) / ny degrees for scalar and U rows and 90 (ny - 2j - 1) / ny
// for V row j; the band edges are decided on those integers exactly.
// Returns 0 (no filter), 1 (simplified filter) or 2 (3-point operator, coefficient in *r).
int filter_band(int num, int ny, double* r) {
  const int m = num < 0 ? -num : num;   // |lat| = 90 m / ny degrees
  *r = 0.0;
  if (m * 90 < 38 * ny) return 1;
  if (m * 90 <= 70 * ny) {
    const double lat = (90.0 * m / ny) * M_PI / 180.0;
    *r = 0.25 * (1.0 - std::cos(lat) / std::cos(38.0 * M_PI / 180.0));
    return 2;
  }
  return 0;
}

template <typename T>
void filter_row(T* F, int nx, int band, double r) {
  if (band == 1) {
    T A(0);
    for (int x = 0; x < nx; ++x) A += (x % 2 == 0) ? F[x] : -F[x];
    A /= double(nx);
    for (int x = 0; x < nx; ++x) F[x] -= (x % 2 == 0) ? A : -A;
  } else if (band == 2) {
    std::vector<T> old(F, F + nx);
    for (int x = 0; x < nx; ++x)
      F[x] = old[x] + r * (old[wrap(x - 1, nx)] - 2.0 * old[x] + old[wrap(x + 1, nx)]);
  }
}

// The filters on every interior row of U, V, Phi and p_s (the pole rows lie poleward of 70 deg).
template <typename T>
void filter_lowlat(const Geo& g, St<T>& y) {
  const Sizes z(g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  double r;
  for (int j = 1; j < ny; ++j) {
    const int band = filter_band(ny - 2 * j, ny, &r);
    for (int k = 0; k < nz; ++k) {
      filter_row(&y.U[z.i3(j, k, 0)], nx, band, r);
      filter_row(&y.F[z.i3(j, k, 0)], nx, band, r);
    }
    filter_row(&y.ps[z.i2(j, 0)], nx, band, r);
  }
  for (int jv = 0; jv < ny; ++jv) {
    const int band = filter_band(ny - 2 * jv - 1, ny, &r);
    for (int k = 0; k < nz; ++k) filter_row(&y.V[z.i3(jv, k, 0)], nx, band, r);
  }
}

// One outer step: msub RK3 sub-steps of the adaptation with dt/msub (3*msub calls),
// then one RK3 step of the advection with dt (3 calls), then (when enabled) the low-latitude
// filters.
template <typename T>
void step(const Geo& g, St<T>& y, double dt, int msub) {
  for (int m = 0; m < msub; ++m) rk3(g, y, dt / msub, 0);
  rk3(g, y, dt, 1);
  if (g.filters) filter_lowlat(g, y);
}

// ---------------------------------------------------------------- adjoint (reverse sweep)
// Adjoint arrays use the same layouts as their forward counterparts.  Every
// statement is the transpose of one forward statement, written scatter style.
struct Adj {
  std::vector<double> pse, Fe, Ue, P, l, q, RT, phi, PU, PV, u, v, MU, MV, D, S, sd, vgl, wp;
};

void adj_alloc(const Geo& g, Adj& b) {
  const Sizes z(g);
  const size_t nvr = (size_t)g.ny * g.nx;
  b.pse.assign(z.n2, 0); b.Fe.assign(z.n3, 0); b.Ue.assign(z.n3, 0);
  b.P.assign(z.n2, 0); b.l.assign(z.n2, 0); b.q.assign(z.n2, 0);
  b.RT.assign(z.n3, 0); b.phi.assign(z.n3, 0); b.PU.assign(z.n2, 0); b.PV.assign(nvr, 0);
  b.u.assign(z.n3, 0); b.MU.assign(z.n3, 0); b.v.assign(z.nv3, 0); b.MV.assign(z.nv3, 0);
  b.D.assign(z.n3, 0); b.S.assign(z.nh3, 0); b.sd.assign(z.nh3, 0);
  b.vgl.assign(z.n3, 0); b.wp.assign(z.n3, 0);
}

// Transpose of diagnose(): consumes b.{wp, vgl, sd, S, D, MU, MV, u, v, PU, PV, phi, RT, P, l, q, Fe, Ue, pse}
// and adds into the state adjoint ay.
void adj_diagnose(const Geo& g, const St<double>& y, const Work<double>& w, Adj& b, St<double>& ay) {
  const Sizes z(g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double a = g.a;

  // omega/p
  for (int j = 0; j <= ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const size_t id = z.i3(j, k, i);
        const double P = w.P[z.i2(j, i)], P2 = P * P;
        const double Sk = w.S[z.ih(j, k, i)] + 0.5 * w.D[id] * g.dsig[k];
        const double aw = b.wp[id];
        b.vgl[id] += aw;
        b.S[z.ih(j, k, i)] += -aw / (g.sig[k] * P2);
        b.D[id] += -0.5 * g.dsig[k] * aw / (g.sig[k] * P2);
        b.P[z.i2(j, i)] += 2.0 * Sk / (g.sig[k] * P2 * P) * aw;
      }

  // v.grad(l), pole rows: zonal mean of the adjacent V-row product, replicated
  for (int k = 0; k < nz; ++k) {
    double an = 0, as = 0;
    for (int i = 0; i < nx; ++i) { an += b.vgl[z.i3(0, k, i)]; as += b.vgl[z.i3(ny, k, i)]; }
    an /= (double(nx) * a * g.dth);
    as /= (double(nx) * a * g.dth);
    for (int i = 0; i < nx; ++i) {
      const double dln = w.l[z.i2(1, i)] - w.l[z.i2(0, i)];
      b.v[z.i3(0, k, i)] += an * dln;
      b.l[z.i2(1, i)] += an * w.v[z.i3(0, k, i)];
      b.l[z.i2(0, i)] -= an * w.v[z.i3(0, k, i)];
      const double dls = w.l[z.i2(ny, i)] - w.l[z.i2(ny - 1, i)];
      b.v[z.i3(ny - 1, k, i)] += as * dls;
      b.l[z.i2(ny, i)] += as * w.v[z.i3(ny - 1, k, i)];
      b.l[z.i2(ny - 1, i)] -= as * w.v[z.i3(ny - 1, k, i)];
    }
  }
  for (int j = 1; j < ny; ++j) {
    const int M = g.M[j], n = g.n[j];
    const double dx = M * a * g.s[j] * g.dlam;
    const double dy = a * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const double av = b.vgl[z.i3(j, k, i)];
        const double dl_r = (w.l[z.i2(j, i + n)] - w.l[z.i2(j, i + 1 - n)]) / dx;
        const double dl_l = (w.l[z.i2(j, i - 1 + n)] - w.l[z.i2(j, i - n)]) / dx;
        b.u[z.i3(j, k, i)] += 0.5 * dl_r * av;
        b.u[z.i3(j, k, i - 1)] += 0.5 * dl_l * av;
        const double adr = 0.5 * w.u[z.i3(j, k, i)] * av / dx;
        const double adl = 0.5 * w.u[z.i3(j, k, i - 1)] * av / dx;
        b.l[z.i2(j, i + n)] += adr;
        b.l[z.i2(j, i + 1 - n)] -= adr;
        b.l[z.i2(j, i - 1 + n)] += adl;
        b.l[z.i2(j, i - n)] -= adl;
        const double am = 0.5 * av / dy;
        b.v[z.i3(j, k, i)] += am * (w.l[z.i2(j + 1, i)] - w.l[z.i2(j, i)]);
        b.l[z.i2(j + 1, i)] += am * w.v[z.i3(j, k, i)];
        b.l[z.i2(j, i)] -= am * w.v[z.i3(j, k, i)];
        b.v[z.i3(j - 1, k, i)] += am * (w.l[z.i2(j, i)] - w.l[z.i2(j - 1, i)]);
        b.l[z.i2(j, i)] += am * w.v[z.i3(j - 1, k, i)];
        b.l[z.i2(j - 1, i)] -= am * w.v[z.i3(j - 1, k, i)];
      }
  }

  // sigma-dot
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const double P = w.P[z.i2(j, i)], P2 = P * P;
      const double Pi = w.S[z.ih(j, nz, i)];
      for (int h = 1; h < nz; ++h) {
        const double as = b.sd[z.ih(j, h, i)];
        b.S[z.ih(j, nz, i)] += g.sigh[h] / P2 * as;
        b.S[z.ih(j, h, i)] += -as / P2;
        b.P[z.i2(j, i)] += -2.0 * (g.sigh[h] * Pi - w.S[z.ih(j, h, i)]) / (P2 * P) * as;
      }
    }

  // prefix sums (S_0 is the constant 0)
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int k = nz - 1; k >= 0; --k) {
        const double as = b.S[z.ih(j, k + 1, i)];
        b.D[z.i3(j, k, i)] += as * g.dsig[k];
        b.S[z.ih(j, k, i)] += as;
      }

  // divergence: poles (replicated cap values), then interior
  for (int k = 0; k < nz; ++k) {
    double an = 0, as = 0;
    for (int i = 0; i < nx; ++i) { an += b.D[z.i3(0, k, i)]; as += b.D[z.i3(ny, k, i)]; }
    for (int i = 0; i < nx; ++i) {
      b.MV[z.i3(0, k, i)] += a * g.dlam * g.sv[0] / g.acap * an;
      b.MV[z.i3(ny - 1, k, i)] += -a * g.dlam * g.sv[ny - 1] / g.acap * as;
    }
  }
  for (int j = 1; j < ny; ++j) {
    const int M = g.M[j], n = g.n[j];
    const double dx = M * a * g.s[j] * g.dlam;
    const double dy = a * g.s[j] * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const double ad = b.D[z.i3(j, k, i)];
        b.MU[z.i3(j, k, i + n - 1)] += ad / dx;
        b.MU[z.i3(j, k, i - n)] -= ad / dx;
        b.MV[z.i3(j, k, i)] += g.sv[j] / dy * ad;
        b.MV[z.i3(j - 1, k, i)] -= g.sv[j - 1] / dy * ad;
      }
  }

  // velocities and mass fluxes
  for (int j = 1; j < ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const size_t id = z.i3(j, k, i);
        const double PU = w.PU[z.i2(j, i)], Ue = w.Ue[id];
        b.Ue[id] += b.u[id] / PU + PU * b.MU[id];
        b.PU[z.i2(j, i)] += -Ue / (PU * PU) * b.u[id] + Ue * b.MU[id];
      }
  for (int jv = 0; jv < ny; ++jv)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const size_t id = z.i3(jv, k, i);
        const double PV = w.PV[z.i2(jv, i)], V = y.V[id];
        ay.V[id] += b.v[id] / PV + PV * b.MV[id];
        b.PV[z.i2(jv, i)] += -V / (PV * PV) * b.v[id] + V * b.MV[id];
      }

  // staggered P
  for (int j = 1; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      b.P[z.i2(j, i)] += 0.5 * b.PU[z.i2(j, i)];
      b.P[z.i2(j, i + 1)] += 0.5 * b.PU[z.i2(j, i)];
    }
  for (int jv = 0; jv < ny; ++jv)
    for (int i = 0; i < nx; ++i) {
      b.P[z.i2(jv, i)] += 0.5 * b.PV[z.i2(jv, i)];
      b.P[z.i2(jv + 1, i)] += 0.5 * b.PV[z.i2(jv, i)];
    }

  // hydrostatic integral: phi_k = cpk_k RT_k + sum_{l>k} cl_l RT_l
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int k = 0; k < nz; ++k) {
        const double ap = b.phi[z.i3(j, k, i)];
        b.RT[z.i3(j, k, i)] += g.cpk[k] * ap;
        for (int l2 = k + 1; l2 < nz; ++l2) b.RT[z.i3(j, l2, i)] += g.cl[l2] * ap;
      }

  // R T' = b Phi / P
  for (int j = 0; j <= ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const size_t id = z.i3(j, k, i);
        const double P = w.P[z.i2(j, i)];
        b.Fe[id] += g.b / P * b.RT[id];
        b.P[z.i2(j, i)] += -g.b * w.Fe[id] / (P * P) * b.RT[id];
      }

  // P, l, q from the pole-read p_s
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t id = z.i2(j, i);
      b.l[id] += b.q[id];
      b.pse[id] += b.P[id] / (2.0 * g.p0 * w.P[id]) + b.l[id] / w.pse[id];
    }

  // U with zero pole rows
  for (int j = 1; j < ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) ay.U[z.i3(j, k, i)] += b.Ue[z.i3(j, k, i)];

  // pole reads: transpose of "replicate the row mean" is "spread the row sum / nx"
  for (int j = 1; j < ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) ay.F[z.i3(j, k, i)] += b.Fe[z.i3(j, k, i)];
  for (int p : {0, ny})
    for (int k = 0; k < nz; ++k) {
      double s = 0;
      for (int i = 0; i < nx; ++i) s += b.Fe[z.i3(p, k, i)];
      for (int i = 0; i < nx; ++i) ay.F[z.i3(p, k, i)] += s / nx;
    }
  for (int j = 1; j < ny; ++j)
    for (int i = 0; i < nx; ++i) ay.ps[z.i2(j, i)] += b.pse[z.i2(j, i)];
  for (int p : {0, ny}) {
    double s = 0;
    for (int i = 0; i < nx; ++i) s += b.pse[z.i2(p, i)];
    for (int i = 0; i < nx; ++i) ay.ps[z.i2(p, i)] += s / nx;
  }
}

// Transpose of tend_A: given at (adjoint of the tendency, full layout), add J^T at into ay.
void adj_tend_A(const Geo& g, const St<double>& y, const Work<double>& w, const St<double>& at, St<double>& ay) {
  const Sizes z(g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double a = g.a, RT0 = g.rd * g.t0;
  Adj b;
  adj_alloc(g, b);

  // V tendency
  for (int jv = 0; jv < ny; ++jv) {
    const double dy = a * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const double atv = at.V[z.i3(jv, k, i)];
        const double dphi = w.phi[z.i3(jv + 1, k, i)] - w.phi[z.i3(jv, k, i)];
        const double dq = w.q[z.i2(jv + 1, i)] - w.q[z.i2(jv, i)];
        const double dl = w.l[z.i2(jv + 1, i)] - w.l[z.i2(jv, i)];
        const double rty = 0.5 * (w.RT[z.i3(jv, k, i)] + w.RT[z.i3(jv + 1, k, i)]);
        const double pgf = (dphi + RT0 * dq + rty * dl) / dy;
        const double UU = 0.25 * (w.Ue[z.i3(jv, k, i - 1)] + w.Ue[z.i3(jv, k, i)] +
                                  w.Ue[z.i3(jv + 1, k, i - 1)] + w.Ue[z.i3(jv + 1, k, i)]);
        const double uu = 0.25 * (w.u[z.i3(jv, k, i - 1)] + w.u[z.i3(jv, k, i)] +
                                  w.u[z.i3(jv + 1, k, i - 1)] + w.u[z.i3(jv + 1, k, i)]);
        const double fs = g.fv[jv] + uu * g.cotv[jv] / a;
        b.PV[z.i2(jv, i)] += -pgf * atv;
        const double gp = -w.PV[z.i2(jv, i)] * atv / dy;
        b.phi[z.i3(jv + 1, k, i)] += gp;
        b.phi[z.i3(jv, k, i)] -= gp;
        b.q[z.i2(jv + 1, i)] += RT0 * gp;
        b.q[z.i2(jv, i)] -= RT0 * gp;
        b.RT[z.i3(jv, k, i)] += 0.5 * dl * gp;
        b.RT[z.i3(jv + 1, k, i)] += 0.5 * dl * gp;
        b.l[z.i2(jv + 1, i)] += rty * gp;
        b.l[z.i2(jv, i)] -= rty * gp;
        const double afs = UU * atv;
        const double auu = 0.25 * g.cotv[jv] / a * afs;
        const double aUU = 0.25 * fs * atv;
        for (int jj : {jv, jv + 1})
          for (int ii : {i - 1, i}) {
            b.u[z.i3(jj, k, ii)] += auu;
            b.Ue[z.i3(jj, k, ii)] += aUU;
          }
      }
  }
  // U tendency
  for (int j = 1; j < ny; ++j) {
    const int M = g.M[j], n = g.n[j];
    const double dx = M * a * g.s[j] * g.dlam;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const double atu = at.U[z.i3(j, k, i)];
        const double dphi = (w.phi[z.i3(j, k, i + n)] - w.phi[z.i3(j, k, i + 1 - n)]) / dx;
        const double dq = (w.q[z.i2(j, i + n)] - w.q[z.i2(j, i + 1 - n)]) / dx;
        const double dl = (w.l[z.i2(j, i + n)] - w.l[z.i2(j, i + 1 - n)]) / dx;
        const double rtx = 0.5 * (w.RT[z.i3(j, k, i)] + w.RT[z.i3(j, k, i + 1)]);
        const double pgf = dphi + RT0 * dq + rtx * dl;
        const double VV = 0.25 * (y.V[z.i3(j, k, i)] + y.V[z.i3(j, k, i + 1)] +
                                  y.V[z.i3(j - 1, k, i)] + y.V[z.i3(j - 1, k, i + 1)]);
        const double fs = g.f[j] + w.u[z.i3(j, k, i)] * g.cot[j] / a;
        b.PU[z.i2(j, i)] += -pgf * atu;
        const double ap = -w.PU[z.i2(j, i)] * atu;
        b.phi[z.i3(j, k, i + n)] += ap / dx;
        b.phi[z.i3(j, k, i + 1 - n)] -= ap / dx;
        b.q[z.i2(j, i + n)] += RT0 * ap / dx;
        b.q[z.i2(j, i + 1 - n)] -= RT0 * ap / dx;
        b.RT[z.i3(j, k, i)] += 0.5 * dl * ap;
        b.RT[z.i3(j, k, i + 1)] += 0.5 * dl * ap;
        b.l[z.i2(j, i + n)] += rtx * ap / dx;
        b.l[z.i2(j, i + 1 - n)] -= rtx * ap / dx;
        b.u[z.i3(j, k, i)] += -VV * atu * g.cot[j] / a;
        const double aVV = -0.25 * fs * atu;
        ay.V[z.i3(j, k, i)] += aVV;
        ay.V[z.i3(j, k, i + 1)] += aVV;
        ay.V[z.i3(j - 1, k, i)] += aVV;
        ay.V[z.i3(j - 1, k, i + 1)] += aVV;
      }
  }
  // p_s tendency
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i) b.S[z.ih(j, nz, i)] += -g.p0 * at.ps[z.i2(j, i)];
  // p_s diffusion (transpose of the flux-form Laplacian, into the pole-read p_s)
  if (g.kstar != 0.0) {
    for (int j = 1; j < ny; ++j) {
      const int M = g.M[j];
      const double dx = M * a * g.s[j] * g.dlam;
      const double dy2 = a * a * g.s[j] * g.dth * g.dth;
      for (int i = 0; i < nx; ++i) {
        const double c = g.kstar * at.ps[z.i2(j, i)];
        b.pse[z.i2(j, i + M)] += c / (dx * dx);
        b.pse[z.i2(j, i - M)] += c / (dx * dx);
        b.pse[z.i2(j, i)] -= 2.0 * c / (dx * dx);
        b.pse[z.i2(j + 1, i)] += c * g.sv[j] / dy2;
        b.pse[z.i2(j, i)] -= c * (g.sv[j] + g.sv[j - 1]) / dy2;
        b.pse[z.i2(j - 1, i)] += c * g.sv[j - 1] / dy2;
      }
    }
    double an = 0, as = 0;
    for (int i = 0; i < nx; ++i) {
      an += g.kstar * at.ps[z.i2(0, i)];
      as += g.kstar * at.ps[z.i2(ny, i)];
    }
    const double cn = g.sv[0] * g.dlam / (g.acap * g.dth), cs = g.sv[ny - 1] * g.dlam / (g.acap * g.dth);
    for (int i = 0; i < nx; ++i) {
      b.pse[z.i2(1, i)] += cn * an;
      b.pse[z.i2(0, i)] -= cn * an;
      b.pse[z.i2(ny - 1, i)] += cs * as;
      b.pse[z.i2(ny, i)] -= cs * as;
    }
  }
  // Phi tendency
  for (int j = 0; j <= ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const size_t id = z.i3(j, k, i);
        const double atf = at.F[id];
        b.P[z.i2(j, i)] += g.b * w.wp[id] * atf;
        b.Fe[id] += g.kappa * w.wp[id] * atf;
        b.wp[id] += (g.b * w.P[z.i2(j, i)] + g.kappa * w.Fe[id]) * atf;
      }
  adj_diagnose(g, y, w, b, ay);
}

// Transpose of tend_L.
void adj_tend_L(const Geo& g, const St<double>& y, const Work<double>& w, const St<double>& at, St<double>& ay) {
  const Sizes z(g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double a = g.a;
  Adj b;
  adj_alloc(g, b);
  std::vector<double> avt(z.nv3, 0.0);

  // V rows
  for (int jv = 0; jv < ny; ++jv) {
    const int M = g.Mv[jv], n = g.nv[jv];
    const double dx2 = 2.0 * M * a * g.sv[jv] * g.dlam;
    const double dy2 = 2.0 * a * g.sv[jv] * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const double am = -at.V[z.i3(jv, k, i)];
        // L1
        {
          const double c1 = am / dx2;
          const double up = 0.5 * (w.u[z.i3(jv, k, i + n - 1)] + w.u[z.i3(jv + 1, k, i + n - 1)]);
          const double um = 0.5 * (w.u[z.i3(jv, k, i - n)] + w.u[z.i3(jv + 1, k, i - n)]);
          const double Vp = y.V[z.i3(jv, k, i + M)], Vm = y.V[z.i3(jv, k, i - M)];
          b.u[z.i3(jv, k, i + n - 1)] += 0.5 * Vp * c1;
          b.u[z.i3(jv + 1, k, i + n - 1)] += 0.5 * Vp * c1;
          ay.V[z.i3(jv, k, i + M)] += up * c1;
          b.u[z.i3(jv, k, i - n)] -= 0.5 * Vm * c1;
          b.u[z.i3(jv + 1, k, i - n)] -= 0.5 * Vm * c1;
          ay.V[z.i3(jv, k, i - M)] -= um * c1;
        }
        // L2 with vts(js) = (vt(js-1)+vt(js))/2 on interior scalar rows
        {
          const double c2 = am / dy2;
          if (jv + 1 < ny) {
            const int js = jv + 1;
            const double vts = 0.5 * (w.v[z.i3(js - 1, k, i)] * g.sv[js - 1] + w.v[z.i3(js, k, i)] * g.sv[js]);
            const double Vn = y.V[z.i3(jv + 1, k, i)];
            avt[z.i3(js - 1, k, i)] += 0.5 * Vn * c2;
            avt[z.i3(js, k, i)] += 0.5 * Vn * c2;
            ay.V[z.i3(jv + 1, k, i)] += vts * c2;
          }
          if (jv > 0) {
            const int js = jv;
            const double vts = 0.5 * (w.v[z.i3(js - 1, k, i)] * g.sv[js - 1] + w.v[z.i3(js, k, i)] * g.sv[js]);
            const double Vs = y.V[z.i3(jv - 1, k, i)];
            avt[z.i3(js - 1, k, i)] -= 0.5 * Vs * c2;
            avt[z.i3(js, k, i)] -= 0.5 * Vs * c2;
            ay.V[z.i3(jv - 1, k, i)] -= vts * c2;
          }
        }
        // L3
        {
          const double c3 = am / (2.0 * g.dsig[k]);
          if (k + 1 < nz) {
            const double sdv = 0.5 * (w.sd[z.ih(jv, k + 1, i)] + w.sd[z.ih(jv + 1, k + 1, i)]);
            const double Vb = y.V[z.i3(jv, k + 1, i)];
            b.sd[z.ih(jv, k + 1, i)] += 0.5 * Vb * c3;
            b.sd[z.ih(jv + 1, k + 1, i)] += 0.5 * Vb * c3;
            ay.V[z.i3(jv, k + 1, i)] += sdv * c3;
          }
          if (k > 0) {
            const double sdv = 0.5 * (w.sd[z.ih(jv, k, i)] + w.sd[z.ih(jv + 1, k, i)]);
            const double Vt = y.V[z.i3(jv, k - 1, i)];
            b.sd[z.ih(jv, k, i)] -= 0.5 * Vt * c3;
            b.sd[z.ih(jv + 1, k, i)] -= 0.5 * Vt * c3;
            ay.V[z.i3(jv, k - 1, i)] -= sdv * c3;
          }
        }
      }
  }
  // U rows
  for (int j = 1; j < ny; ++j) {
    const int M = g.M[j], n = g.n[j];
    const double dx2 = 2.0 * M * a * g.s[j] * g.dlam;
    const double dy2 = 2.0 * a * g.s[j] * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const double am = -at.U[z.i3(j, k, i)];
        {
          const double c1 = am / dx2;
          const double ubp = 0.5 * (w.u[z.i3(j, k, i + n - 1)] + w.u[z.i3(j, k, i + n)]);
          const double ubm = 0.5 * (w.u[z.i3(j, k, i - n)] + w.u[z.i3(j, k, i + 1 - n)]);
          const double Up = w.Ue[z.i3(j, k, i + M)], Um = w.Ue[z.i3(j, k, i - M)];
          b.u[z.i3(j, k, i + n - 1)] += 0.5 * Up * c1;
          b.u[z.i3(j, k, i + n)] += 0.5 * Up * c1;
          b.Ue[z.i3(j, k, i + M)] += ubp * c1;
          b.u[z.i3(j, k, i - n)] -= 0.5 * Um * c1;
          b.u[z.i3(j, k, i + 1 - n)] -= 0.5 * Um * c1;
          b.Ue[z.i3(j, k, i - M)] -= ubm * c1;
        }
        {
          const double c2 = am / dy2;
          const double vn = 0.5 * (w.v[z.i3(j, k, i)] * g.sv[j] + w.v[z.i3(j, k, i + 1)] * g.sv[j]);
          const double vs = 0.5 * (w.v[z.i3(j - 1, k, i)] * g.sv[j - 1] + w.v[z.i3(j - 1, k, i + 1)] * g.sv[j - 1]);
          const double Un = w.Ue[z.i3(j + 1, k, i)], Us = w.Ue[z.i3(j - 1, k, i)];
          avt[z.i3(j, k, i)] += 0.5 * Un * c2;
          avt[z.i3(j, k, i + 1)] += 0.5 * Un * c2;
          b.Ue[z.i3(j + 1, k, i)] += vn * c2;
          avt[z.i3(j - 1, k, i)] -= 0.5 * Us * c2;
          avt[z.i3(j - 1, k, i + 1)] -= 0.5 * Us * c2;
          b.Ue[z.i3(j - 1, k, i)] -= vs * c2;
        }
        {
          const double c3 = am / (2.0 * g.dsig[k]);
          if (k + 1 < nz) {
            const double sdu = 0.5 * (w.sd[z.ih(j, k + 1, i)] + w.sd[z.ih(j, k + 1, i + 1)]);
            const double Ub = w.Ue[z.i3(j, k + 1, i)];
            b.sd[z.ih(j, k + 1, i)] += 0.5 * Ub * c3;
            b.sd[z.ih(j, k + 1, i + 1)] += 0.5 * Ub * c3;
            b.Ue[z.i3(j, k + 1, i)] += sdu * c3;
          }
          if (k > 0) {
            const double sdu = 0.5 * (w.sd[z.ih(j, k, i)] + w.sd[z.ih(j, k, i + 1)]);
            const double Ut = w.Ue[z.i3(j, k - 1, i)];
            b.sd[z.ih(j, k, i)] -= 0.5 * Ut * c3;
            b.sd[z.ih(j, k, i + 1)] -= 0.5 * Ut * c3;
            b.Ue[z.i3(j, k - 1, i)] -= sdu * c3;
          }
        }
      }
  }
  // Phi, interior rows
  for (int j = 1; j < ny; ++j) {
    const int M = g.M[j], n = g.n[j];
    const double dx2 = 2.0 * M * a * g.s[j] * g.dlam;
    const double dy2 = 2.0 * a * g.s[j] * g.dth;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const double am = -at.F[z.i3(j, k, i)];
        {
          const double c1 = am / dx2;
          b.u[z.i3(j, k, i + n - 1)] += w.Fe[z.i3(j, k, i + M)] * c1;
          b.Fe[z.i3(j, k, i + M)] += w.u[z.i3(j, k, i + n - 1)] * c1;
          b.u[z.i3(j, k, i - n)] -= w.Fe[z.i3(j, k, i - M)] * c1;
          b.Fe[z.i3(j, k, i - M)] -= w.u[z.i3(j, k, i - n)] * c1;
        }
        {
          const double c2 = am / dy2;
          avt[z.i3(j, k, i)] += w.Fe[z.i3(j + 1, k, i)] * c2;
          b.Fe[z.i3(j + 1, k, i)] += w.v[z.i3(j, k, i)] * g.sv[j] * c2;
          avt[z.i3(j - 1, k, i)] -= w.Fe[z.i3(j - 1, k, i)] * c2;
          b.Fe[z.i3(j - 1, k, i)] -= w.v[z.i3(j - 1, k, i)] * g.sv[j - 1] * c2;
        }
        {
          const double c3 = am / (2.0 * g.dsig[k]);
          if (k + 1 < nz) {
            b.sd[z.ih(j, k + 1, i)] += w.Fe[z.i3(j, k + 1, i)] * c3;
            b.Fe[z.i3(j, k + 1, i)] += w.sd[z.ih(j, k + 1, i)] * c3;
          }
          if (k > 0) {
            b.sd[z.ih(j, k, i)] -= w.Fe[z.i3(j, k - 1, i)] * c3;
            b.Fe[z.i3(j, k - 1, i)] -= w.sd[z.ih(j, k, i)] * c3;
          }
        }
      }
  }
  // Phi, pole rows (the cap sum is taken once per replicated copy)
  const double cc = a * g.dlam / (2.0 * g.acap);
  for (int k = 0; k < nz; ++k) {
    for (int p : {0, ny}) {
      double asum = 0;
      for (int i = 0; i < nx; ++i) {
        const double am = -at.F[z.i3(p, k, i)];
        asum += am;
        const double c3 = am / (2.0 * g.dsig[k]);
        if (k + 1 < nz) {
          b.sd[z.ih(p, k + 1, i)] += w.Fe[z.i3(p, k + 1, i)] * c3;
          b.Fe[z.i3(p, k + 1, i)] += w.sd[z.ih(p, k + 1, i)] * c3;
        }
        if (k > 0) {
          b.sd[z.ih(p, k, i)] -= w.Fe[z.i3(p, k - 1, i)] * c3;
          b.Fe[z.i3(p, k - 1, i)] -= w.sd[z.ih(p, k, i)] * c3;
        }
      }
      const int jv = (p == 0) ? 0 : ny - 1;
      const int js = (p == 0) ? 1 : ny - 1;
      const double sg = (p == 0) ? cc : -cc;
      for (int i = 0; i < nx; ++i) {
        avt[z.i3(jv, k, i)] += sg * w.Fe[z.i3(js, k, i)] * asum;
        b.Fe[z.i3(js, k, i)] += sg * w.v[z.i3(jv, k, i)] * g.sv[jv] * asum;
      }
    }
  }
  // vt = v * sin(theta_v)
  for (int jv = 0; jv < ny; ++jv)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) b.v[z.i3(jv, k, i)] += g.sv[jv] * avt[z.i3(jv, k, i)];
  adj_diagnose(g, y, w, b, ay);
}

void adj_tendency(const Geo& g, const St<double>& y, int which, const St<double>& at, St<double>& ay) {
  Work<double> w;
  diagnose(g, y, w);
  if (which == 0) adj_tend_A(g, y, w, at, ay); else adj_tend_L(g, y, w, at, ay);
}

// Transpose of stage(): aout -> (abase, ayin), added into the given accumulators.
void adj_stage(const Geo& g, const St<double>& yin, double ch, int which, const St<double>& aout,
               St<double>& abase, St<double>& ayin) {
  const Sizes z(g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  St<double> at;
  at.U.assign(z.n3, 0); at.V.assign(z.nv3, 0); at.F.assign(z.n3, 0); at.ps.assign(z.n2, 0);
  for (int j = 1; j < ny; ++j)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const size_t id = z.i3(j, k, i);
        abase.U[id] += aout.U[id];
        at.U[id] = ch * aout.U[id];
      }
  for (size_t id = 0; id < z.nv3; ++id) { abase.V[id] += aout.V[id]; at.V[id] = ch * aout.V[id]; }
  for (size_t id = 0; id < z.n3; ++id) at.F[id] = ch * aout.F[id];
  for (size_t id = 0; id < z.n2; ++id) at.ps[id] = ch * aout.ps[id];
  for (int j = 1; j < ny; ++j) {
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) abase.F[z.i3(j, k, i)] += aout.F[z.i3(j, k, i)];
    for (int i = 0; i < nx; ++i) abase.ps[z.i2(j, i)] += aout.ps[z.i2(j, i)];
  }
  for (int p : {0, ny}) {
    double s = 0;
    for (int i = 0; i < nx; ++i) s += aout.ps[z.i2(p, i)];
    for (int i = 0; i < nx; ++i) abase.ps[z.i2(p, i)] += s / nx;
    for (int k = 0; k < nz; ++k) {
      double sf = 0;
      for (int i = 0; i < nx; ++i) sf += aout.F[z.i3(p, k, i)];
      for (int i = 0; i < nx; ++i) abase.F[z.i3(p, k, i)] += sf / nx;
    }
  }
  adj_tendency(g, yin, which, at, ayin);
}

void zero_like(const Geo& g, St<double>& s) {
  const Sizes z(g);
  s.U.assign(z.n3, 0); s.V.assign(z.nv3, 0); s.F.assign(z.n3, 0); s.ps.assign(z.n2, 0);
}

// Transpose of rk3 about its start state y: a (adjoint of y+) -> adjoint of y.
void adj_rk3(const Geo& g, const St<double>& y, double h, int which, St<double>& a) {
  St<double> y1, y2;
  stage(g, y, y, h / 3.0, which, y1);
  stage(g, y, y1, h / 2.0, which, y2);
  St<double> ay, ay1, ay2;
  zero_like(g, ay); zero_like(g, ay1); zero_like(g, ay2);
  adj_stage(g, y2, h, which, a, ay, ay2);
  adj_stage(g, y1, h / 2.0, which, ay2, ay, ay1);
  adj_stage(g, y, h / 3.0, which, ay1, ay, ay);
  a = ay;
}

// Transpose of step about its start state y0.
void adj_step(const Geo& g, const St<double>& y0, double dt, int msub, St<double>& a) {
  // the filters act last and each row operator is symmetric: their transpose is themselves
  if (g.filters) filter_lowlat(g, a);
  std::vector<St<double>> starts;
  St<double> y = y0;
  for (int m = 0; m < msub; ++m) { starts.push_back(y); rk3(g, y, dt / msub, 0); }
  adj_rk3(g, y, dt, 1, a);
  for (int m = msub - 1; m >= 0; --m) adj_rk3(g, starts[m], dt / msub, 0, a);
}

// ---------------------------------------------------------------- geometry
Geo* make_geo(int nx, int ny, int nz, const double* sigma_half, const double* phis, const double* consts) {
  Geo* g = new Geo();
  g->nx = nx; g->ny = ny; g->nz = nz;
  // Constants: a, Omega, g, R, c_p, p0, T0 (consts may override, 0 keeps the default)
  double c[7] = {6.371e6, 7.292e-5, 9.80616, 287.04, 1004.64, 1.0e5, 300.0};
  if (consts) for (int i = 0; i < 7; ++i) if (consts[i] != 0.0) c[i] = consts[i];
  g->a = c[0]; g->omega = c[1]; g->g = c[2]; g->rd = c[3]; g->cp = c[4]; g->p0 = c[5]; g->t0 = c[6];
  g->kappa = g->rd / g->cp;
  g->b = std::sqrt(g->kappa * g->rd * g->t0);
  g->dlam = 2.0 * M_PI / nx;
  g->dth = M_PI / ny;
  g->acap = 2.0 * M_PI * g->a * g->a * (1.0 - std::cos(0.5 * g->dth));
  g->s.assign(ny + 1, 0); g->cot.assign(ny + 1, 0); g->f.assign(ny + 1, 0);
  g->r.assign(ny + 1, 0); g->M.assign(ny + 1, 1); g->n.assign(ny + 1, 1);
  for (int j = 1; j < ny; ++j) {
    const double th = j * g->dth;
    g->s[j] = std::sin(th);
    g->cot[j] = std::cos(th) / std::sin(th);
    g->f[j] = 2.0 * g->omega * std::cos(th);
    g->M[j] = leap_span(g->s[j], g->dlam, nx, &g->r[j]);
    g->n[j] = (g->M[j] + 1) / 2;
  }
  g->sv.assign(ny, 0); g->cotv.assign(ny, 0); g->fv.assign(ny, 0);
  g->rv.assign(ny, 0); g->Mv.assign(ny, 1); g->nv.assign(ny, 1);
  for (int jv = 0; jv < ny; ++jv) {
    const double th = (jv + 0.5) * g->dth;
    g->sv[jv] = std::sin(th);
    g->cotv[jv] = std::cos(th) / std::sin(th);
    g->fv[jv] = 2.0 * g->omega * std::cos(th);
    g->Mv[jv] = leap_span(g->sv[jv], g->dlam, nx, &g->rv[jv]);
    g->nv[jv] = (g->Mv[jv] + 1) / 2;
  }
  g->sigh.assign(nz + 1, 0);
  for (int h = 0; h <= nz; ++h) g->sigh[h] = sigma_half ? sigma_half[h] : double(h) / nz;
  g->sig.assign(nz, 0); g->dsig.assign(nz, 0); g->cl.assign(nz, 0); g->cpk.assign(nz, 0);
  for (int k = 0; k < nz; ++k) {
    g->sig[k] = 0.5 * (g->sigh[k] + g->sigh[k + 1]);
    g->dsig[k] = g->sigh[k + 1] - g->sigh[k];
    g->cl[k] = (k >= 1) ? std::log(g->sigh[k + 1] / g->sigh[k]) : 0.0;
    g->cpk[k] = std::log(g->sigh[k + 1] / g->sig[k]);
  }
  g->phis.assign((size_t)(ny + 1) * nx, 0.0);
  if (phis) std::memcpy(g->phis.data(), phis, sizeof(double) * (ny + 1) * nx);
  for (int p : {0, ny}) {
    double m = 0;
    for (int i = 0; i < nx; ++i) m += g->phis[(size_t)p * nx + i];
    m /= nx;
    for (int i = 0; i < nx; ++i) g->phis[(size_t)p * nx + i] = m;
  }
  return g;
}

template <typename T>
void load(const Geo& g, St<T>& s, const double* U, const double* V, const double* F, const double* ps) {
  const Sizes z(g);
  s.U.assign(U, U + z.n3); s.V.assign(V, V + z.nv3); s.F.assign(F, F + z.n3); s.ps.assign(ps, ps + z.n2);
}

void store(const Geo& g, const St<double>& s, double* U, double* V, double* F, double* ps) {
  const Sizes z(g);
  std::memcpy(U, s.U.data(), sizeof(double) * z.n3);
  std::memcpy(V, s.V.data(), sizeof(double) * z.nv3);
  std::memcpy(F, s.F.data(), sizeof(double) * z.n3);
  std::memcpy(ps, s.ps.data(), sizeof(double) * z.n2);
}

}  // namespace

// ================================================================ C ABI for the tests
extern "C" {

void* orc_create(int nx, int ny, int nz, const double* sigma_half, const double* phis, const double* consts) {
  if (nx < 8 || ny < 4 || nz < 1) return nullptr;
  return make_geo(nx, ny, nz, sigma_half, phis, consts);
}

void orc_destroy(void* h) { delete static_cast<Geo*>(h); }

// Threads the OpenMP loops of the forward map use (the adjoint sweep is serial).
int orc_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Sets the thread count of the forward map's OpenMP loops (for timing at 1 and at all threads).
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// Physical constants in use: a, Omega, g, R, c_p, p0, T0, kappa, b, A_cap
void orc_constants(void* h, double* out) {
  const Geo& g = *static_cast<Geo*>(h);
  const double v[10] = {g.a, g.omega, g.g, g.rd, g.cp, g.p0, g.t0, g.kappa, g.b, g.acap};
  std::memcpy(out, v, sizeof(v));
}

// Leap table: span M (odd) per scalar/U row (ny+1, poles 1) and per V row (ny),
// and the raw eq. 7 ratios before rounding.
void orc_leap_table(void* h, int* m_rows, int* m_vrows, double* r_rows, double* r_vrows) {
  const Geo& g = *static_cast<Geo*>(h);
  for (int j = 0; j <= g.ny; ++j) { if (m_rows) m_rows[j] = g.M[j]; if (r_rows) r_rows[j] = g.r[j]; }
  for (int j = 0; j < g.ny; ++j) { if (m_vrows) m_vrows[j] = g.Mv[j]; if (r_vrows) r_vrows[j] = g.rv[j]; }
}

// Zonal grid spacing a sin(theta) dlam of each scalar/U row and each V row (metres).
void orc_zonal_spacing(void* h, double* dx_rows, double* dx_vrows) {
  const Geo& g = *static_cast<Geo*>(h);
  for (int j = 0; j <= g.ny; ++j) dx_rows[j] = g.a * std::sin(j * g.dth) * g.dlam;
  for (int j = 0; j < g.ny; ++j) dx_vrows[j] = g.a * g.sv[j] * g.dlam;
}

// Tendency of one process (which = 0 adaptation A, 1 advection -L), full layouts,
// pole rows replicated, U pole rows zero.
void orc_tendency(void* h, int which, const double* U, const double* V, const double* F, const double* ps,
                  double* tU, double* tV, double* tF, double* tps) {
  const Geo& g = *static_cast<Geo*>(h);
  St<double> y, t;
  load(g, y, U, V, F, ps);
  tendency(g, y, which, t);
  store(g, t, tU, tV, tF, tps);
}

// Column diagnostics of a state: D, phi', omega/p, v.grad(l) (scalar 3D), sigma-dot at half
// levels, Pi (2D).  Any output pointer may be NULL.
void orc_column_diag(void* h, const double* U, const double* V, const double* F, const double* ps,
                     double* D, double* phi, double* wp, double* sd, double* Pi, double* vgl) {
  const Geo& g = *static_cast<Geo*>(h);
  const Sizes z(g);
  St<double> y;
  load(g, y, U, V, F, ps);
  Work<double> w;
  diagnose(g, y, w);
  if (D) std::memcpy(D, w.D.data(), sizeof(double) * z.n3);
  if (phi) std::memcpy(phi, w.phi.data(), sizeof(double) * z.n3);
  if (wp) std::memcpy(wp, w.wp.data(), sizeof(double) * z.n3);
  if (sd) std::memcpy(sd, w.sd.data(), sizeof(double) * z.nh3);
  if (vgl) std::memcpy(vgl, w.vgl.data(), sizeof(double) * z.n3);
  if (Pi)
    for (int j = 0; j <= g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) Pi[z.i2(j, i)] = w.S[z.ih(j, g.nz, i)];
}

// One stage out = base + ch * T(yin).
void orc_stage(void* h, int which, double ch,
               const double* bU, const double* bV, const double* bF, const double* bps,
               const double* U, const double* V, const double* F, const double* ps,
               double* oU, double* oV, double* oF, double* ops) {
  const Geo& g = *static_cast<Geo*>(h);
  St<double> base, yin, out;
  load(g, base, bU, bV, bF, bps);
  load(g, yin, U, V, F, ps);
  stage(g, base, yin, ch, which, out);
  store(g, out, oU, oV, oF, ops);
}

// nsteps outer steps in place.
void orc_step(void* h, double* U, double* V, double* F, double* ps, int nsteps, double dt, int msub) {
  const Geo& g = *static_cast<Geo*>(h);
  St<double> y;
  load(g, y, U, V, F, ps);
  for (int s = 0; s < nsteps; ++s) step(g, y, dt, msub);
  store(g, y, U, V, F, ps);
}

// Tangent-linear of nsteps outer steps by complex step: out = d step(y)[dy] (exact to rounding).
void orc_tl_step_cs(void* h, const double* U, const double* V, const double* F, const double* ps,
                    const double* dU, const double* dV, const double* dF, const double* dps,
                    double* oU, double* oV, double* oF, double* ops, int nsteps, double dt, int msub) {
  const Geo& g = *static_cast<Geo*>(h);
  const Sizes z(g);
  const double hc = 1e-30;
  St<cplx> y;
  y.U.resize(z.n3); y.V.resize(z.nv3); y.F.resize(z.n3); y.ps.resize(z.n2);
  for (size_t i = 0; i < z.n3; ++i) { y.U[i] = cplx(U[i], hc * dU[i]); y.F[i] = cplx(F[i], hc * dF[i]); }
  for (size_t i = 0; i < z.nv3; ++i) y.V[i] = cplx(V[i], hc * dV[i]);
  for (size_t i = 0; i < z.n2; ++i) y.ps[i] = cplx(ps[i], hc * dps[i]);
  for (int s = 0; s < nsteps; ++s) step(g, y, dt, msub);
  for (size_t i = 0; i < z.n3; ++i) { oU[i] = y.U[i].imag() / hc; oF[i] = y.F[i].imag() / hc; }
  for (size_t i = 0; i < z.nv3; ++i) oV[i] = y.V[i].imag() / hc;
  for (size_t i = 0; i < z.n2; ++i) ops[i] = y.ps[i].imag() / hc;
}

// Tangent-linear of one tendency by complex step.
void orc_tl_tendency_cs(void* h, int which, const double* U, const double* V, const double* F, const double* ps,
                        const double* dU, const double* dV, const double* dF, const double* dps,
                        double* oU, double* oV, double* oF, double* ops) {
  const Geo& g = *static_cast<Geo*>(h);
  const Sizes z(g);
  const double hc = 1e-30;
  St<cplx> y, t;
  y.U.resize(z.n3); y.V.resize(z.nv3); y.F.resize(z.n3); y.ps.resize(z.n2);
  for (size_t i = 0; i < z.n3; ++i) { y.U[i] = cplx(U[i], hc * dU[i]); y.F[i] = cplx(F[i], hc * dF[i]); }
  for (size_t i = 0; i < z.nv3; ++i) y.V[i] = cplx(V[i], hc * dV[i]);
  for (size_t i = 0; i < z.n2; ++i) y.ps[i] = cplx(ps[i], hc * dps[i]);
  tendency(g, y, which, t);
  for (size_t i = 0; i < z.n3; ++i) { oU[i] = t.U[i].imag() / hc; oF[i] = t.F[i].imag() / hc; }
  for (size_t i = 0; i < z.nv3; ++i) oV[i] = t.V[i].imag() / hc;
  for (size_t i = 0; i < z.n2; ++i) ops[i] = t.ps[i].imag() / hc;
}

// Adjoint of one tendency about y: (aU..) in = adjoint of the tendency; out arrays receive J^T a.
void orc_adj_tendency(void* h, int which, const double* U, const double* V, const double* F, const double* ps,
                      const double* aU, const double* aV, const double* aF, const double* aps,
                      double* oU, double* oV, double* oF, double* ops) {
  const Geo& g = *static_cast<Geo*>(h);
  St<double> y, at, ay;
  load(g, y, U, V, F, ps);
  load(g, at, aU, aV, aF, aps);
  zero_like(g, ay);
  adj_tendency(g, y, which, at, ay);
  store(g, ay, oU, oV, oF, ops);
}

// Adjoint of one stage out = base + ch * T(in) about `in`: the adjoint of base and of in.
void orc_adj_stage(void* h, int which, double ch, const double* U, const double* V, const double* F, const double* ps,
                   const double* aU, const double* aV, const double* aF, const double* aps,
                   double* bU, double* bV, double* bF, double* bps, double* iU, double* iV, double* iF, double* ips) {
  const Geo& g = *static_cast<Geo*>(h);
  St<double> y, ao, ab, ai;
  load(g, y, U, V, F, ps);
  load(g, ao, aU, aV, aF, aps);
  zero_like(g, ab);
  zero_like(g, ai);
  adj_stage(g, y, ch, which, ao, ab, ai);
  store(g, ab, bU, bV, bF, bps);
  store(g, ai, iU, iV, iF, ips);
}

// Adjoint of one outer step about its start state (U0..): a in = adjoint of the output,
// a out = adjoint of the input (in place).
void orc_adj_step(void* h, const double* U0, const double* V0, const double* F0, const double* ps0,
                  double* aU, double* aV, double* aF, double* aps, double dt, int msub) {
  const Geo& g = *static_cast<Geo*>(h);
  St<double> y, a;
  load(g, y, U0, V0, F0, ps0);
  load(g, a, aU, aV, aF, aps);
  adj_step(g, y, dt, msub, a);
  store(g, a, aU, aV, aF, aps);
}

// Global mass sum_j w_j sum_i p_s + A_cap (p_N + p_S) and the quadratic energy measure.
void orc_diagnostics(void* h, const double* U, const double* V, const double* F, const double* ps,
                     double* mass, double* energy) {
  const Geo& g = *static_cast<Geo*>(h);
  const Sizes z(g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double a2 = g.a * g.a;
  double m = 0, e = 0, es = 0;
  double pn = 0, psn = 0;
  for (int i = 0; i < nx; ++i) { pn += ps[z.i2(0, i)]; psn += ps[z.i2(ny, i)]; }
  pn /= nx; psn /= nx;
  for (int j = 1; j < ny; ++j) {
    const double w = a2 * g.s[j] * g.dth * g.dlam;
    for (int i = 0; i < nx; ++i) m += w * ps[z.i2(j, i)];
  }
  m += g.acap * (pn + psn);
  // energy: (p0 / 2g) sum w dsig (U^2 + V^2 + Phi^2) + (R T0 p0 / 2g) sum w q^2
  for (int j = 1; j < ny; ++j) {
    const double w = a2 * g.s[j] * g.dth * g.dlam;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const double uu = U[z.i3(j, k, i)], ff = F[z.i3(j, k, i)];
        e += w * g.dsig[k] * (uu * uu + ff * ff);
      }
    for (int i = 0; i < nx; ++i) {
      const double q = std::log(ps[z.i2(j, i)] / g.p0) + g.phis[z.i2(j, i)] / (g.rd * g.t0);
      es += w * q * q;
    }
  }
  for (int jv = 0; jv < ny; ++jv) {
    const double w = a2 * g.sv[jv] * g.dth * g.dlam;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) { const double vv = V[z.i3(jv, k, i)]; e += w * g.dsig[k] * vv * vv; }
  }
  for (int p : {0, ny}) {
    for (int k = 0; k < nz; ++k) {
      double fm = 0;
      for (int i = 0; i < nx; ++i) fm += F[z.i3(p, k, i)];
      fm /= nx;
      e += g.acap * g.dsig[k] * fm * fm;
    }
    const double pm = (p == 0) ? pn : psn;
    const double q = std::log(pm / g.p0) + g.phis[z.i2(p, 0)] / (g.rd * g.t0);
    es += g.acap * q * q;
  }
  *mass = m;
  *energy = g.p0 / (2.0 * g.g) * e + g.rd * g.t0 * g.p0 / (2.0 * g.g) * es;
}

// Low-latitude filters on (step) or off; the state filter alone, in place.
void orc_set_filters(void* h, int on) { static_cast<Geo*>(h)->filters = on ? 1 : 0; }

// p_s diffusion coefficient kappa* of eq. 1 (m^2/s; 0 = off).
void orc_set_kstar(void* h, double kstar) { static_cast<Geo*>(h)->kstar = kstar; }

void orc_filter(void* h, double* U, double* V, double* F, double* ps) {
  const Geo& g = *static_cast<Geo*>(h);
  St<double> y;
  load(g, y, U, V, F, ps);
  filter_lowlat(g, y);
  store(g, y, U, V, F, ps);
}

// Sub-step count from the CFL rule: ceil(omega_max dt / (0.8 sqrt 3)) with
// omega_max = 2 c sqrt(1/dx45^2 + 1/dy^2), c = 350 m/s.
int orc_substeps(void* h, double dt) {
  const Geo& g = *static_cast<Geo*>(h);
  const double dx45 = g.a * std::cos(M_PI / 4.0) * g.dlam;
  const double dy = g.a * g.dth;
  const double wmax = 2.0 * 350.0 * std::sqrt(1.0 / (dx45 * dx45) + 1.0 / (dy * dy));
  int m = (int)std::ceil(wmax * dt / (0.8 * std::sqrt(3.0)));
  return m < 1 ? 1 : m;
}

}  // extern "C"
