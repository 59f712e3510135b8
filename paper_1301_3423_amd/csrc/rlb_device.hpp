// Device-side building blocks of one lattice update of the third-order
// relativistic lattice Boltzmann scheme (Sec. II D, Eq. rlb:disc).
//
// Every lattice point i is a compile-time constant: its integer displacement
// theta_i, its shell energy p0_i and its weight w_i come from the quadrature
// table compiled into the library.  Loops over points are unrolled at compile
// time, so theta components and weights become instruction immediates and
// zero components cost nothing.  Points are stored in inversion pairs
// (2k, 2k+1) with theta_{2k+1} = -theta_{2k}, sorted by shell.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace rlb {

struct Point {
  int tx, ty, tz, shell;
  double p0, w;
};

inline constexpr Point D3Q128[128] = {
#include "../lattice/d3q128.inc"
};

// Inverse Gram matrix of the 30 light-cone monomials (gen_constants.py).
inline constexpr double GINV[30][30] = {
#include "rlb_ginv.inc"
};

inline constexpr int Q = 128;
inline constexpr int NPAIR = Q / 2;
inline constexpr int NSHELL = 4;
inline constexpr int R2 = 41;
inline constexpr double R = 0x1.99ccc999fff00p+2;      // sqrt(41)
inline constexpr double INV_R = 0x1.3fd8077e70577p-3;  // 1/sqrt(41)
inline constexpr double INV_R2 = 0x1.8f9c18f9c18fap-6; // 1/41
inline constexpr double INV_R3 = 0x1.f344ba86edcd2p-9; // 1/41^(3/2)
inline constexpr int MAXD = 6;                         // max |theta component|

inline constexpr unsigned FLAG_NONFINITE = 1u;
inline constexpr unsigned FLAG_NONPHYSICAL = 2u;
inline constexpr unsigned FLAG_LANDAU = 4u;

// ---- compile-time facts about the table --------------------------------

constexpr bool table_is_paired() {
  for (int k = 0; k < NPAIR; ++k) {
    const Point &a = D3Q128[2 * k], &b = D3Q128[2 * k + 1];
    if (a.tx != -b.tx || a.ty != -b.ty || a.tz != -b.tz) return false;
    if (a.shell != b.shell || a.p0 != b.p0 || a.w != b.w) return false;
    if (a.tx * a.tx + a.ty * a.ty + a.tz * a.tz != R2) return false;
  }
  for (int i = 1; i < Q; ++i)
    if (D3Q128[i].shell < D3Q128[i - 1].shell) return false;
  return true;
}
static_assert(table_is_paired(), "quadrature table must be inversion-paired and shell-sorted");

constexpr int shell_pair_begin(int l) {
  for (int k = 0; k < NPAIR; ++k)
    if (D3Q128[2 * k].shell >= l) return k;
  return NPAIR;
}
constexpr double shell_p0(int l) { return D3Q128[2 * shell_pair_begin(l)].p0; }

// Fused multiply-add in the precision of its operands (the double builtin
// would silently promote float arithmetic).
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// ---- lattice geometry and the gather offsets ----------------------------

struct Geom {
  int nx, ny, nz;
  int cells;      // nx * ny * nz
  int64_t stride; // elements between consecutive populations
};

// (c - s) mod n for |s| <= MAXD; n is uniform across the wavefront.
__device__ __forceinline__ int wrap_back(int c, int s, int n) {
  if (n > MAXD) {
    int t = c - s;
    if (s > 0) t += (t < 0) ? n : 0;
    if (s < 0) t -= (t >= n) ? n : 0;
    return t;
  }
  if (n == 1) return 0;
  return (c - s + (MAXD + 1) * n) % n;
}

// Offsets (in elements, within one population array) of the cells
// x - s for every shift s in [-6, 6] along each axis; the compiler keeps
// only the shifts the table uses.
struct Shifts {
  int xo[2 * MAXD + 1], yo[2 * MAXD + 1], zo[2 * MAXD + 1];
  __device__ __forceinline__ Shifts(int x, int y, int z, const Geom &g) {
#pragma unroll
    for (int s = -MAXD; s <= MAXD; ++s) {
      xo[s + MAXD] = wrap_back(x, s, g.nx);
      yo[s + MAXD] = wrap_back(y, s, g.ny) * g.nx;
      zo[s + MAXD] = wrap_back(z, s, g.nz) * (g.nx * g.ny);
    }
  }
  // cell x - theta (the source of a pull) for compile-time theta
  template <int TX, int TY, int TZ>
  __device__ __forceinline__ int back() const {
    return zo[TZ + MAXD] + yo[TY + MAXD] + xo[TX + MAXD];
  }
  // cell x + theta (the destination of a push)
  template <int TX, int TY, int TZ>
  __device__ __forceinline__ int fwd() const {
    return zo[MAXD - TZ] + yo[MAXD - TY] + xo[MAXD - TX];
  }
};

// ---- moments (step 1) ----------------------------------------------------

struct Moments {
  double N0, Nx, Ny, Nz;
  double T00, T0x, T0y, T0z, Txx, Tyy, Tzz, Txy, Txz, Tyz;
};

// N^mu = sum_i f_i p_i^mu and T^{mu nu} = sum_i f_i p_i^mu p_i^nu, using
// the pairs: with s = f_i + f_inv(i) and d = f_i - f_inv(i), the even
// moments take s and the odd ones d.  Sums per shell carry integer theta
// factors; the energy and R powers are applied once per shell.  Always
// accumulated in float64.
template <class S>
__device__ __forceinline__ Moments moments(const S (&f)[Q]) {
  Moments m{};
  static_for<0, NSHELL>([&](auto L) {
    constexpr int l = decltype(L)::value;
    constexpr int kb = shell_pair_begin(l), ke = shell_pair_begin(l + 1);
    double sh = 0, sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0, dx = 0, dy = 0, dz = 0;
    static_for<kb, ke>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr Point P = D3Q128[2 * k];
      const double a = static_cast<double>(f[2 * k]);
      const double b = static_cast<double>(f[2 * k + 1]);
      const double s = a + b, d = a - b;
      sh += s;
      if constexpr (P.tx != 0) sxx = __builtin_fma(double(P.tx * P.tx), s, sxx);
      if constexpr (P.ty != 0) syy = __builtin_fma(double(P.ty * P.ty), s, syy);
      if constexpr (P.tz != 0) szz = __builtin_fma(double(P.tz * P.tz), s, szz);
      if constexpr (P.tx * P.ty != 0) sxy = __builtin_fma(double(P.tx * P.ty), s, sxy);
      if constexpr (P.tx * P.tz != 0) sxz = __builtin_fma(double(P.tx * P.tz), s, sxz);
      if constexpr (P.ty * P.tz != 0) syz = __builtin_fma(double(P.ty * P.tz), s, syz);
      if constexpr (P.tx != 0) dx = __builtin_fma(double(P.tx), d, dx);
      if constexpr (P.ty != 0) dy = __builtin_fma(double(P.ty), d, dy);
      if constexpr (P.tz != 0) dz = __builtin_fma(double(P.tz), d, dz);
      // finish this pair before the next: otherwise the even chains are sunk
      // to the end of the shell and every s stays live (an empty statement
      // that reads and writes the accumulators; it emits no instruction)
      asm volatile("" : "+v"(sh), "+v"(sxx), "+v"(syy), "+v"(szz), "+v"(sxy), "+v"(sxz), "+v"(syz), "+v"(dx),
                   "+v"(dy), "+v"(dz));
    });
    constexpr double p = shell_p0(l);
    constexpr double p1r = p * INV_R, p2 = p * p, p2r = p * p * INV_R, p2r2 = p * p * INV_R2;
    m.N0 = __builtin_fma(p, sh, m.N0);
    m.T00 = __builtin_fma(p2, sh, m.T00);
    m.Nx = __builtin_fma(p1r, dx, m.Nx);
    m.Ny = __builtin_fma(p1r, dy, m.Ny);
    m.Nz = __builtin_fma(p1r, dz, m.Nz);
    m.T0x = __builtin_fma(p2r, dx, m.T0x);
    m.T0y = __builtin_fma(p2r, dy, m.T0y);
    m.T0z = __builtin_fma(p2r, dz, m.T0z);
    m.Txx = __builtin_fma(p2r2, sxx, m.Txx);
    m.Tyy = __builtin_fma(p2r2, syy, m.Tyy);
    m.Tzz = __builtin_fma(p2r2, szz, m.Tzz);
    m.Txy = __builtin_fma(p2r2, sxy, m.Txy);
    m.Txz = __builtin_fma(p2r2, sxz, m.Txz);
    m.Tyz = __builtin_fma(p2r2, syz, m.Tyz);
  });
  return m;
}

// ---- Landau-Lifshitz frame (steps 2-3) -----------------------------------

struct Frame {
  double n, eps, T;
  double U0, Ux, Uy, Uz; // U^mu = gamma (1, v)
  double vx, vy, vz;
};

// Solves T^{mu nu} U_nu = eps U^mu for the timelike eigenvector
// (Eq. eigenproblem).  With U = gamma (1, v), E = T^00, M = T^{0i} and
// S = T^{ij} the eigenproblem is equivalent to
//   r(v) = (E - M.v) v - (M - S v) = 0,   eps = E - M.v,
// solved here by Newton's method with Jacobian (E - M.v) I - v M^T + S,
// started from the exact solution for an ideal fluid with P = eps/3:
// |v0| = 3x / (2 + sqrt(4 - 3x^2)) along M, x = |M|/E.
// Then n = U_mu N^mu and T = eps / (3 n).  Returns RLB flags.
__device__ __forceinline__ unsigned landau_frame(const Moments &m, Frame &fr) {
  const double E = m.T00, Mx = m.T0x, My = m.T0y, Mz = m.T0z;
  const double Sxx = m.Txx, Syy = m.Tyy, Szz = m.Tzz, Sxy = m.Txy, Sxz = m.Txz, Syz = m.Tyz;
  const double Mabs = __builtin_sqrt(Mx * Mx + My * My + Mz * Mz);
  const double x = Mabs / E;
  const double disc = __builtin_fmax(4.0 - 3.0 * x * x, 0.0);
  const double v0 = 3.0 * x / (2.0 + __builtin_sqrt(disc));
  const double sc = (Mabs > 0.0) ? v0 / Mabs : 0.0;
  double vx = Mx * sc, vy = My * sc, vz = Mz * sc;
  bool converged = false;
  for (int it = 0; it < 24; ++it) {
    const double a = E - (Mx * vx + My * vy + Mz * vz);
    const double rx = a * vx - Mx + (Sxx * vx + Sxy * vy + Sxz * vz);
    const double ry = a * vy - My + (Sxy * vx + Syy * vy + Syz * vz);
    const double rz = a * vz - Mz + (Sxz * vx + Syz * vy + Szz * vz);
    const double j00 = a - vx * Mx + Sxx, j01 = -vx * My + Sxy, j02 = -vx * Mz + Sxz;
    const double j10 = -vy * Mx + Sxy, j11 = a - vy * My + Syy, j12 = -vy * Mz + Syz;
    const double j20 = -vz * Mx + Sxz, j21 = -vz * My + Syz, j22 = a - vz * Mz + Szz;
    const double c00 = j11 * j22 - j12 * j21, c01 = j12 * j20 - j10 * j22, c02 = j10 * j21 - j11 * j20;
    const double c10 = j02 * j21 - j01 * j22, c11 = j00 * j22 - j02 * j20, c12 = j01 * j20 - j00 * j21;
    const double c20 = j01 * j12 - j02 * j11, c21 = j02 * j10 - j00 * j12, c22 = j00 * j11 - j01 * j10;
    const double inv_det = 1.0 / (j00 * c00 + j01 * c01 + j02 * c02);
    const double dx = (c00 * rx + c10 * ry + c20 * rz) * inv_det;
    const double dy = (c01 * rx + c11 * ry + c21 * rz) * inv_det;
    const double dz = (c02 * rx + c12 * ry + c22 * rz) * inv_det;
    vx -= dx;
    vy -= dy;
    vz -= dz;
    const double dmax = __builtin_fmax(__builtin_fabs(dx), __builtin_fmax(__builtin_fabs(dy), __builtin_fabs(dz)));
    const double vmax = __builtin_fmax(__builtin_fabs(vx), __builtin_fmax(__builtin_fabs(vy), __builtin_fabs(vz)));
    if (dmax <= 1e-12 * vmax || dmax < 1e-300) {
      converged = true;
      break;
    }
  }
  unsigned flags = converged ? 0u : FLAG_LANDAU;
  const double v2 = vx * vx + vy * vy + vz * vz;
  const double eps = E - (Mx * vx + My * vy + Mz * vz);
  const double gamma = 1.0 / __builtin_sqrt(1.0 - v2);
  const double n = gamma * (m.N0 - (vx * m.Nx + vy * m.Ny + vz * m.Nz));
  if (!(v2 < 1.0) || !(n > 0.0) || !(eps > 0.0)) flags |= FLAG_NONPHYSICAL;
  if (!__builtin_isfinite(n + eps + gamma)) flags |= FLAG_NONFINITE;
  fr.n = n;
  fr.eps = eps;
  fr.T = eps / (3.0 * n);
  fr.U0 = gamma;
  fr.Ux = gamma * vx;
  fr.Uy = gamma * vy;
  fr.Uz = gamma * vz;
  fr.vx = vx;
  fr.vy = vy;
  fr.vz = vz;
  return flags;
}

// ---- relaxation time (step 4) ---------------------------------------------

struct Relax {
  int mode;     // 0 fixed, 1 from eta/s
  double tau;   // fixed value
  double eta_s; // ratio eta/s
};

__device__ __forceinline__ double relaxation_time(const Relax &r, double n, double T) {
  if (r.mode == 0) return r.tau;
  return 0.5 + (1.5 * R / T) * r.eta_s * (4.0 - log(n / (T * T * T)));
}

// ---- equilibrium (step 5) ---------------------------------------------------

// Coefficients c of the projected Maxwell-Juttner distribution in the
// monomial basis: c = G^-1 M, with M the moments of the continuous
// distribution (Z = n/(2T), N = nU, T = nT(4UU - eta),
// P = 4nT^2(6UUU - eta U - eta U - eta U)) of each monomial.  G^-1 is block
// diagonal by the parity class of the monomials, so M is formed one block
// at a time (at most eight values live).
struct EqCoef {
  double c[30];
};

inline constexpr int CLASS_BEGIN[9] = {0, 8, 13, 18, 23, 25, 27, 29, 30};

struct MJ {
  double n, a, b, U0, Ux, Uy, Uz, Z; // a = nT, b = 4 n T^2, Z = n/(2T)
  template <int IDX>
  __device__ __forceinline__ double moment() const {
    if constexpr (IDX == 0) return Z;
    else if constexpr (IDX == 1) return n * U0;
    else if constexpr (IDX == 2) return a * (4.0 * U0 * U0 - 1.0);
    else if constexpr (IDX == 3) return b * U0 * (6.0 * U0 * U0 - 3.0);
    else if constexpr (IDX == 4) return a * (4.0 * Ux * Ux + 1.0);
    else if constexpr (IDX == 5) return a * (4.0 * Uy * Uy + 1.0);
    else if constexpr (IDX == 6) return b * U0 * (6.0 * Ux * Ux + 1.0);
    else if constexpr (IDX == 7) return b * U0 * (6.0 * Uy * Uy + 1.0);
    else if constexpr (IDX == 8) return n * Ux;
    else if constexpr (IDX == 9) return 4.0 * a * U0 * Ux;
    else if constexpr (IDX == 10) return b * Ux * (6.0 * U0 * U0 - 1.0);
    else if constexpr (IDX == 11) return b * Ux * (6.0 * Ux * Ux + 3.0);
    else if constexpr (IDX == 12) return b * Ux * (6.0 * Uy * Uy + 1.0);
    else if constexpr (IDX == 13) return n * Uy;
    else if constexpr (IDX == 14) return 4.0 * a * U0 * Uy;
    else if constexpr (IDX == 15) return b * Uy * (6.0 * U0 * U0 - 1.0);
    else if constexpr (IDX == 16) return b * Uy * (6.0 * Ux * Ux + 1.0);
    else if constexpr (IDX == 17) return b * Uy * (6.0 * Uy * Uy + 3.0);
    else if constexpr (IDX == 18) return n * Uz;
    else if constexpr (IDX == 19) return 4.0 * a * U0 * Uz;
    else if constexpr (IDX == 20) return b * Uz * (6.0 * U0 * U0 - 1.0);
    else if constexpr (IDX == 21) return b * Uz * (6.0 * Ux * Ux + 1.0);
    else if constexpr (IDX == 22) return b * Uz * (6.0 * Uy * Uy + 1.0);
    else if constexpr (IDX == 23) return 4.0 * a * Ux * Uy;
    else if constexpr (IDX == 24) return 6.0 * b * U0 * Ux * Uy;
    else if constexpr (IDX == 25) return 4.0 * a * Ux * Uz;
    else if constexpr (IDX == 26) return 6.0 * b * U0 * Ux * Uz;
    else if constexpr (IDX == 27) return 4.0 * a * Uy * Uz;
    else if constexpr (IDX == 28) return 6.0 * b * U0 * Uy * Uz;
    else return 6.0 * b * Ux * Uy * Uz;
  }
};

__device__ __forceinline__ EqCoef eq_coefficients(double n, double T, double U0, double Ux, double Uy,
                                                  double Uz) {
  const MJ mj{n, n * T, 4.0 * n * T * T, U0, Ux, Uy, Uz, n / (2.0 * T)};
  EqCoef e;
  static_for<0, 8>([&](auto B) {
    constexpr int blk = decltype(B)::value;
    constexpr int b0 = CLASS_BEGIN[blk], b1 = CLASS_BEGIN[blk + 1];
    double M[b1 - b0];
    static_for<b0, b1>([&](auto J) {
      constexpr int j = decltype(J)::value;
      M[j - b0] = mj.template moment<j>();
    });
    static_for<b0, b1>([&](auto A) {
      constexpr int ia = decltype(A)::value;
      double acc = 0.0;
      static_for<b0, b1>([&](auto J) {
        constexpr int j = decltype(J)::value;
        if constexpr (GINV[ia][j] != 0.0) acc = __builtin_fma(GINV[ia][j], M[j - b0], acc);
      });
      e.c[ia] = acc;
    });
  });
  return e;
}

// The equilibrium on one energy shell p = p0_l as a cubic polynomial of the
// integer direction theta:  h = E(theta) + O(theta), even and odd parts,
//   E = A + Bxx tx^2 + Byy ty^2 + Bxy tx ty + Bxz tx tz + Byz ty tz
//   O = Cx tx + Cy ty + Cz tz + D111 tx^3 + D122 tx ty^2 + D112 tx^2 ty
//       + D222 ty^3 + D113 tx^2 tz + D223 ty^2 tz + D123 tx ty tz,
// so that f_i^eq = w_i (E + O) and f_inv(i)^eq = w_i (E - O).
template <class CT>
struct ShellCoef {
  CT A, Bxx, Byy, Bxy, Bxz, Byz;
  CT Cx, Cy, Cz, D111, D122, D112, D222, D113, D223, D123;
};

template <int L, class CT>
__device__ __forceinline__ ShellCoef<CT> shell_coefficients(const EqCoef &e) {
  constexpr double p = shell_p0(L);
  constexpr double q2 = p * p * INV_R2, q3 = p * p * p * INV_R2, r1 = p * INV_R, r2 = p * p * INV_R,
                   r3 = p * p * p * INV_R, d3 = p * p * p * INV_R3;
  const double *c = e.c;
  ShellCoef<CT> s;
  s.A = CT(__builtin_fma(p, __builtin_fma(p, __builtin_fma(p, c[3], c[2]), c[1]), c[0]));
  s.Bxx = CT(__builtin_fma(q3, c[6], q2 * c[4]));
  s.Byy = CT(__builtin_fma(q3, c[7], q2 * c[5]));
  s.Bxy = CT(__builtin_fma(q3, c[24], q2 * c[23]));
  s.Bxz = CT(__builtin_fma(q3, c[26], q2 * c[25]));
  s.Byz = CT(__builtin_fma(q3, c[28], q2 * c[27]));
  s.Cx = CT(__builtin_fma(r3, c[10], __builtin_fma(r2, c[9], r1 * c[8])));
  s.Cy = CT(__builtin_fma(r3, c[15], __builtin_fma(r2, c[14], r1 * c[13])));
  s.Cz = CT(__builtin_fma(r3, c[20], __builtin_fma(r2, c[19], r1 * c[18])));
  s.D111 = CT(d3 * c[11]);
  s.D122 = CT(d3 * c[12]);
  s.D112 = CT(d3 * c[16]);
  s.D222 = CT(d3 * c[17]);
  s.D113 = CT(d3 * c[21]);
  s.D223 = CT(d3 * c[22]);
  s.D123 = CT(d3 * c[29]);
  return s;
}

template <int IDX, class CT>
__device__ __forceinline__ void shell_eval(const ShellCoef<CT> &s, CT &Ev, CT &Od) {
  constexpr int tx = D3Q128[IDX].tx, ty = D3Q128[IDX].ty, tz = D3Q128[IDX].tz;
  CT E = s.A;
  if constexpr (tx != 0) E = fmadd(CT(tx * tx), s.Bxx, E);
  if constexpr (ty != 0) E = fmadd(CT(ty * ty), s.Byy, E);
  if constexpr (tx * ty != 0) E = fmadd(CT(tx * ty), s.Bxy, E);
  if constexpr (tx * tz != 0) E = fmadd(CT(tx * tz), s.Bxz, E);
  if constexpr (ty * tz != 0) E = fmadd(CT(ty * tz), s.Byz, E);
  CT O = CT(0);
  if constexpr (tx != 0) O = fmadd(CT(tx), s.Cx, O);
  if constexpr (ty != 0) O = fmadd(CT(ty), s.Cy, O);
  if constexpr (tz != 0) O = fmadd(CT(tz), s.Cz, O);
  if constexpr (tx != 0) O = fmadd(CT(tx * tx * tx), s.D111, O);
  if constexpr (tx * ty != 0) O = fmadd(CT(tx * ty * ty), s.D122, O);
  if constexpr (tx * ty != 0) O = fmadd(CT(tx * tx * ty), s.D112, O);
  if constexpr (ty != 0) O = fmadd(CT(ty * ty * ty), s.D222, O);
  if constexpr (tx * tz != 0) O = fmadd(CT(tx * tx * tz), s.D113, O);
  if constexpr (ty * tz != 0) O = fmadd(CT(ty * ty * tz), s.D223, O);
  if constexpr (tx * ty * tz != 0) O = fmadd(CT(tx * ty * tz), s.D123, O);
  Ev = E;
  Od = O;
}

} // namespace rlb
