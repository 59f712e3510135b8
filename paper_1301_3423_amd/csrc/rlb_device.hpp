// Device-side building blocks of one lattice update of the relativistic
// lattice Boltzmann scheme (Sec. II D, Eq. rlb:disc), generic over the model:
//   Model<3>: the third-order model, R = sqrt(41), 128 points on 4 energy
//             shells, equilibrium on the 30 polynomials of Table I
//             (Eq. equi3rd);
//   Model<2>: the second-order model of Appendix A, R = 3, 66 points on 3
//             energy shells, equilibrium on the 14 polynomials of degree
//             <= 2 (Eq. equi2nd).
//
// Every lattice point i is a compile-time constant: its integer displacement
// theta_i, its shell energy p0_i and its weight w_i come from the quadrature
// tables compiled into the library.  Loops over points are unrolled at
// compile time, so theta components and weights become instruction
// immediates and zero components cost nothing.  Points are stored in
// inversion pairs (2k, 2k+1) with theta_{2k+1} = -theta_{2k}, sorted by shell.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace rlb {

struct Point {
  int tx, ty, tz, shell;
  double p0, w;
};

// exponents of p0, px, py, pz in one monomial of an equilibrium basis
struct Mono {
  int a0, ax, ay, az;
};

template <int ORDER>
struct Model;

// Basis order and blocks follow gen_constants.py, which writes the exact
// inverse Gram matrices: monomials grouped by the parity of their spatial
// exponents (G is block diagonal), pz^2 left out (pz^2 = p0^2 - px^2 - py^2
// on the light cone).
template <>
struct Model<3> {
  static constexpr int ORDER = 3;
  static constexpr int Q = 128;
  static constexpr int NSHELL = 4;
  static constexpr int R2 = 41;
  static constexpr double R = 0x1.99ccc999fff00p+2;      // sqrt(41)
  static constexpr double INV_R = 0x1.3fd8077e70577p-3;  // 1/sqrt(41)
  static constexpr double INV_R2 = 0x1.8f9c18f9c18fap-6; // 1/41
  static constexpr double INV_R3 = 0x1.f344ba86edcd2p-9; // 1/41^(3/2)
  // shear viscosity eta = n T (tau - 1/2) / (VISC R)   (Sec. III)
  static constexpr double VISC = 1.5;
  static constexpr Point P[Q] = {
#include "../lattice/d3q128.inc"
  };
  static constexpr int NM = 30;
  static constexpr Mono MONO[NM] = {
      {0, 0, 0, 0}, {1, 0, 0, 0}, {2, 0, 0, 0}, {3, 0, 0, 0}, {0, 2, 0, 0}, {0, 0, 2, 0}, {1, 2, 0, 0},
      {1, 0, 2, 0}, {0, 1, 0, 0}, {1, 1, 0, 0}, {2, 1, 0, 0}, {0, 3, 0, 0}, {0, 1, 2, 0}, {0, 0, 1, 0},
      {1, 0, 1, 0}, {2, 0, 1, 0}, {0, 2, 1, 0}, {0, 0, 3, 0}, {0, 0, 0, 1}, {1, 0, 0, 1}, {2, 0, 0, 1},
      {0, 2, 0, 1}, {0, 0, 2, 1}, {0, 1, 1, 0}, {1, 1, 1, 0}, {0, 1, 0, 1}, {1, 1, 0, 1}, {0, 0, 1, 1},
      {1, 0, 1, 1}, {0, 1, 1, 1}};
  static constexpr int NBLOCK = 8;
  static constexpr int BLOCK_BEGIN[NBLOCK + 1] = {0, 8, 13, 18, 23, 25, 27, 29, 30};
  static constexpr double GINV[NM][NM] = {
#include "rlb_ginv3.inc"
  };
};

template <>
struct Model<2> {
  static constexpr int ORDER = 2;
  static constexpr int Q = 66;
  static constexpr int NSHELL = 3;
  static constexpr int R2 = 9;
  static constexpr double R = 3.0;
  static constexpr double INV_R = 1.0 / 3.0;
  static constexpr double INV_R2 = 1.0 / 9.0;
  static constexpr double INV_R3 = 1.0 / 27.0;
  // eta_2nd = n T (tau - 1/2) / (7 R), the fit of Appendix A
  static constexpr double VISC = 7.0;
  static constexpr Point P[Q] = {
#include "../lattice/d3q66.inc"
  };
  static constexpr int NM = 14;
  static constexpr Mono MONO[NM] = {{0, 0, 0, 0}, {1, 0, 0, 0}, {2, 0, 0, 0}, {0, 2, 0, 0}, {0, 0, 2, 0},
                                    {0, 1, 0, 0}, {1, 1, 0, 0}, {0, 0, 1, 0}, {1, 0, 1, 0}, {0, 0, 0, 1},
                                    {1, 0, 0, 1}, {0, 1, 1, 0}, {0, 1, 0, 1}, {0, 0, 1, 1}};
  static constexpr int NBLOCK = 7;
  static constexpr int BLOCK_BEGIN[NBLOCK + 1] = {0, 5, 7, 9, 11, 12, 13, 14};
  static constexpr double GINV[NM][NM] = {
#include "rlb_ginv2.inc"
  };
};

using M3 = Model<3>;
using M2 = Model<2>;

inline constexpr int MAXD = 6; // largest |theta component| of either table

inline constexpr unsigned FLAG_NONFINITE = 1u;
inline constexpr unsigned FLAG_NONPHYSICAL = 2u;
inline constexpr unsigned FLAG_LANDAU = 4u;

// ---- compile-time facts about a table ------------------------------------

template <class M>
constexpr bool table_is_paired() {
  for (int k = 0; k < M::Q / 2; ++k) {
    const Point &a = M::P[2 * k], &b = M::P[2 * k + 1];
    if (a.tx != -b.tx || a.ty != -b.ty || a.tz != -b.tz) return false;
    if (a.shell != b.shell || a.p0 != b.p0 || a.w != b.w) return false;
    if (a.tx * a.tx + a.ty * a.ty + a.tz * a.tz != M::R2) return false;
    if (a.tx > MAXD || -a.tx > MAXD || a.ty > MAXD || -a.ty > MAXD || a.tz > MAXD || -a.tz > MAXD) return false;
  }
  for (int i = 1; i < M::Q; ++i)
    if (M::P[i].shell < M::P[i - 1].shell) return false;
  return M::P[M::Q - 1].shell == M::NSHELL - 1;
}
static_assert(table_is_paired<M3>(), "third-order table must be inversion-paired and shell-sorted");
static_assert(table_is_paired<M2>(), "second-order table must be inversion-paired and shell-sorted");

template <class M>
constexpr int shell_pair_begin(int l) {
  for (int k = 0; k < M::Q / 2; ++k)
    if (M::P[2 * k].shell >= l) return k;
  return M::Q / 2;
}
template <class M>
constexpr double shell_p0(int l) {
  return M::P[2 * shell_pair_begin<M>(l)].p0;
}

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
  int cells; // nx * ny * nz
};

// ---- storage of the populations: tiles --------------------------------------
//
// Populations are stored in tiles of TILE = 256 / sizeof(S) consecutive
// cells (32 in float64, 64 in float32).  A tile holds population 0 of its
// cells (256 bytes), then population 1, ..., population Q-1, so population i
// of cell c is element
//     (c / TILE) * Q * TILE + i * TILE + c % TILE
// of a buffer.  A block of the step kernels then reads and writes a few
// contiguous tiles instead of 128 separate arrays: measured on a load/store
// probe with the step's access pattern at 256^3, 2.95 ms per step against
// 3.24 ms with one array per population in float32, 6.25 ms against 7.0 ms
// in float64.
template <class S>
inline constexpr int TILE = 256 / static_cast<int>(sizeof(S));

// Element of population 0 of cell c >= 0 (population i adds i * TILE).
template <class M, class S>
__device__ __forceinline__ int64_t tile_elem(int c) {
  constexpr unsigned T = TILE<S>;
  const unsigned u = static_cast<unsigned>(c);
  return static_cast<int64_t>(u / T) * (M::Q * T) + (u % T);
}

// The same for the x part of a cell inside a row that starts on a tile
// boundary (nx a multiple of TILE): 32-bit, below nx * Q.
template <class M, class S>
__device__ __forceinline__ int tile_elem_x(int x) {
  constexpr unsigned T = TILE<S>;
  const unsigned u = static_cast<unsigned>(x);
  return static_cast<int>((u / T) * (M::Q * T) + (u % T));
}

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

// Integer-weighted sums over the pairs of one shell: sh = sum s,
// sab = sum theta_a theta_b s, da = sum theta_a d, with s = f_i + f_inv(i)
// and d = f_i - f_inv(i).
struct ShellSums {
  double sh, sxx, syy, szz, sxy, sxz, syz, dx, dy, dz;

  template <class M, int K>
  __device__ __forceinline__ void add_pair(double s, double d) {
    constexpr Point P = M::P[2 * K];
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
  }
  // Finish this pair before the next: otherwise the compiler sinks the even
  // chains to the end of the shell and every s stays live.  An empty
  // statement that reads and writes the accumulators; it emits nothing.
  __device__ __forceinline__ void pin() {
    asm volatile("" : "+v"(sh), "+v"(sxx), "+v"(syy), "+v"(szz), "+v"(sxy), "+v"(sxz), "+v"(syz), "+v"(dx),
                 "+v"(dy), "+v"(dz));
  }
  // Folds the sums of shell L into the moments: the energy and R powers of
  // the shell are applied once.
  template <class M, int L>
  __device__ __forceinline__ void fold(Moments &m) const {
    constexpr double p = shell_p0<M>(L);
    constexpr double p1r = p * M::INV_R, p2 = p * p, p2r = p * p * M::INV_R, p2r2 = p * p * M::INV_R2;
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
  }
};

// N^mu = sum_i f_i p_i^mu and T^{mu nu} = sum_i f_i p_i^mu p_i^nu with
// p_i = p0_i (1, theta_i / R), from the pair sums of each shell.  Always
// accumulated in float64.
template <class M, class S>
__device__ __forceinline__ Moments moments(const S (&f)[M::Q]) {
  Moments m{};
  static_for<0, M::NSHELL>([&](auto L) {
    constexpr int l = decltype(L)::value;
    ShellSums a{};
    static_for<shell_pair_begin<M>(l), shell_pair_begin<M>(l + 1)>([&](auto K) {
      constexpr int k = decltype(K)::value;
      const double x = static_cast<double>(f[2 * k]);
      const double y = static_cast<double>(f[2 * k + 1]);
      a.template add_pair<M, k>(x + y, x - y);
      a.pin();
    });
    a.template fold<M, l>(m);
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
// |v0| = 3x / (2 + sqrt(4 - 3x^2)) along M, x = |M|/E.  It stops when the
// update is below 1e-12 of |v|, or one iteration earlier once convergence is
// quadratic: after updates d_prev and d with d <= d_prev / 100, the next
// update would be about d^3 / d_prev^2, and below 1e-14 |v| it is not taken
// (from the ideal-fluid start this saves the last of the usual three
// iterations).  Then n = U_mu N^mu and T = eps / (3 n).  Returns RLB flags.
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
  double dprev = 0.0;
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
    const bool settled = it > 0 && dmax <= 0.01 * dprev && dmax * dmax * dmax <= 1e-14 * vmax * dprev * dprev;
    if (dmax <= 1e-12 * vmax || dmax < 1e-300 || settled) {
      converged = true;
      break;
    }
    dprev = dmax;
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

// From eta = n T (tau - 1/2) / (VISC R) and the entropy density
// s = 4 n - n ln(n / T^3):  tau = 1/2 + (VISC R / T) (eta/s) (4 - ln(n/T^3)).
template <class M>
__device__ __forceinline__ double relaxation_time(const Relax &r, double n, double T) {
  if (r.mode == 0) return r.tau;
  return 0.5 + (M::VISC * M::R / T) * r.eta_s * (4.0 - log(n / (T * T * T)));
}

// ---- equilibrium (step 5) ---------------------------------------------------

// Coefficients c of the projected Maxwell-Juttner distribution in the
// monomial basis: c = G^-1 M, with M the moments of the continuous
// distribution of each basis monomial.  G^-1 is block diagonal by the
// parity class of the monomials, so M is formed one block at a time (at
// most eight values live).
template <class M>
struct EqCoef {
  double c[M::NM];
};

// Moments of the Maxwell-Juttner distribution for the equation of state
// eps = 3 n T:  Z = n/(2T) for the constant monomial, N^mu = n U^mu,
// T^{mu nu} = n T (4 U^mu U^nu - eta^{mu nu}) and
// P^{mu nu lambda} = 4 n T^2 (6 U U U - eta U - eta U - eta U) (symmetrised),
// with eta = diag(1, -1, -1, -1).
struct MJ {
  double n, a, b, Z; // a = nT, b = 4 n T^2, Z = n/(2T)
  double u[4];       // U^mu

  static constexpr double eta(int i, int j) { return i != j ? 0.0 : (i == 0 ? 1.0 : -1.0); }

  // the moment of the monomial p0^A0 px^AX py^AY pz^AZ
  template <int A0, int AX, int AY, int AZ>
  __device__ __forceinline__ double moment() const {
    constexpr int D = A0 + AX + AY + AZ;
    // the tensor indices of the monomial in ascending order
    constexpr int i = A0 > 0 ? 0 : (A0 + AX > 0 ? 1 : (A0 + AX + AY > 0 ? 2 : 3));
    constexpr int j = A0 > 1 ? 0 : (A0 + AX > 1 ? 1 : (A0 + AX + AY > 1 ? 2 : 3));
    constexpr int k = A0 > 2 ? 0 : (A0 + AX > 2 ? 1 : (A0 + AX + AY > 2 ? 2 : 3));
    if constexpr (D == 0) {
      return Z;
    } else if constexpr (D == 1) {
      return n * u[i];
    } else if constexpr (D == 2) {
      if constexpr (eta(i, j) != 0.0)
        return a * (4.0 * u[i] * u[j] - eta(i, j));
      else
        return 4.0 * a * u[i] * u[j];
    } else {
      static_assert(D == 3, "equilibrium monomials have degree <= 3");
      constexpr double e = eta(i, j) + eta(i, k) + eta(j, k);
      // at most one pair of equal indices unless all three are equal
      if constexpr (i == j && j == k)
        return b * u[i] * (6.0 * u[i] * u[i] - 3.0 * eta(i, i));
      else if constexpr (eta(i, j) != 0.0)
        return b * u[k] * (6.0 * u[i] * u[j] - eta(i, j));
      else if constexpr (eta(j, k) != 0.0)
        return b * u[i] * (6.0 * u[j] * u[k] - eta(j, k));
      else if constexpr (eta(i, k) != 0.0)
        return b * u[j] * (6.0 * u[i] * u[k] - eta(i, k));
      else {
        static_assert(e == 0.0);
        return 6.0 * b * u[i] * u[j] * u[k];
      }
    }
  }
};

template <class M>
__device__ __forceinline__ EqCoef<M> eq_coefficients(double n, double T, double U0, double Ux, double Uy,
                                                     double Uz) {
  const MJ mj{n, n * T, 4.0 * n * T * T, n / (2.0 * T), {U0, Ux, Uy, Uz}};
  EqCoef<M> e;
  static_for<0, M::NBLOCK>([&](auto B) {
    constexpr int blk = decltype(B)::value;
    constexpr int b0 = M::BLOCK_BEGIN[blk], b1 = M::BLOCK_BEGIN[blk + 1];
    double Mb[b1 - b0];
    static_for<b0, b1>([&](auto J) {
      constexpr int j = decltype(J)::value;
      constexpr Mono mo = M::MONO[j];
      Mb[j - b0] = mj.template moment<mo.a0, mo.ax, mo.ay, mo.az>();
    });
    static_for<b0, b1>([&](auto A) {
      constexpr int ia = decltype(A)::value;
      double acc = 0.0;
      static_for<b0, b1>([&](auto J) {
        constexpr int j = decltype(J)::value;
        if constexpr (M::GINV[ia][j] != 0.0) acc = __builtin_fma(M::GINV[ia][j], Mb[j - b0], acc);
      });
      e.c[ia] = acc;
    });
  });
  return e;
}

// On shell l (p0 = p), the basis monomial (a0, ax, ay, az) equals
// p^(a0+ax+ay+az) R^-(ax+ay+az) tx^ax ty^ay tz^az, so the equilibrium there
// is a polynomial in the integer direction theta whose coefficient of
// tx^ax ty^ay tz^az collects the basis coefficients with that spatial part.
// SPATIAL<M> lists the distinct spatial parts of the basis in order of
// first appearance (16 for the third-order basis, 9 for the second-order).
constexpr bool same_spatial(const Mono &a, const Mono &b) { return a.ax == b.ax && a.ay == b.ay && a.az == b.az; }

template <class M>
constexpr int spatial_count() {
  int n = 0;
  for (int j = 0; j < M::NM; ++j) {
    bool seen = false;
    for (int i = 0; i < j; ++i) seen = seen || same_spatial(M::MONO[i], M::MONO[j]);
    n += seen ? 0 : 1;
  }
  return n;
}

template <class M>
struct SpatialTable {
  static constexpr int NS = spatial_count<M>();
  Mono part[NS]; // a0 unused
  int of[M::NM]; // spatial index of each basis monomial
};

template <class M>
constexpr SpatialTable<M> make_spatial() {
  SpatialTable<M> t{};
  int n = 0;
  for (int j = 0; j < M::NM; ++j) {
    int found = -1;
    for (int s = 0; s < n; ++s)
      if (same_spatial(t.part[s], M::MONO[j])) found = s;
    if (found < 0) {
      t.part[n] = Mono{0, M::MONO[j].ax, M::MONO[j].ay, M::MONO[j].az};
      found = n++;
    }
    t.of[j] = found;
  }
  return t;
}

template <class M>
inline constexpr SpatialTable<M> SPATIAL = make_spatial<M>();

template <class M, class CT>
struct ShellCoef {
  CT c[SpatialTable<M>::NS];
};

constexpr double ipow(double x, int e) { return e == 0 ? 1.0 : x * ipow(x, e - 1); }
constexpr int ipow(int x, int e) { return e == 0 ? 1 : x * ipow(x, e - 1); }

template <class M>
constexpr double inv_r_pow(int e) {
  return e == 0 ? 1.0 : e == 1 ? M::INV_R : e == 2 ? M::INV_R2 : M::INV_R3;
}

// Coefficients of the theta-polynomial of shell L, rounded once to CT.
// The terms of one spatial part are accumulated from the highest energy
// power down.
template <class M, int L, class CT>
__device__ __forceinline__ ShellCoef<M, CT> shell_coefficients(const EqCoef<M> &e) {
  constexpr double p = shell_p0<M>(L);
  ShellCoef<M, CT> s;
  static_for<0, SpatialTable<M>::NS>([&](auto Sx) {
    constexpr int si = decltype(Sx)::value;
    double acc = 0.0;
    static_for<0, M::NM>([&](auto J) {
      constexpr int j = M::NM - 1 - decltype(J)::value;
      if constexpr (SPATIAL<M>.of[j] == si) {
        constexpr Mono mo = M::MONO[j];
        constexpr int sd = mo.ax + mo.ay + mo.az;
        constexpr double k = ipow(p, mo.a0 + sd) * inv_r_pow<M>(sd);
        acc = __builtin_fma(k, e.c[j], acc);
      }
    });
    s.c[si] = CT(acc);
  });
  return s;
}

// Even (E) and odd (O) parts of the theta-polynomial at point IDX, so that
// f_IDX^eq = w (E + O) and f_inv(IDX)^eq = w (E - O).
template <class M, int IDX, class CT>
__device__ __forceinline__ void shell_eval(const ShellCoef<M, CT> &s, CT &Ev, CT &Od) {
  constexpr Point P = M::P[IDX];
  CT E = s.c[0]; // spatial part 0 is the constant
  static_assert(SPATIAL<M>.part[0].ax + SPATIAL<M>.part[0].ay + SPATIAL<M>.part[0].az == 0);
  CT O = CT(0);
  static_for<1, SpatialTable<M>::NS>([&](auto Sx) {
    constexpr int si = decltype(Sx)::value;
    constexpr Mono sp = SPATIAL<M>.part[si];
    constexpr int mono = ipow(P.tx, sp.ax) * ipow(P.ty, sp.ay) * ipow(P.tz, sp.az);
    if constexpr (mono != 0) {
      if constexpr ((sp.ax + sp.ay + sp.az) % 2 == 0)
        E = fmadd(CT(mono), s.c[si], E);
      else
        O = fmadd(CT(mono), s.c[si], O);
    }
  });
  Ev = E;
  Od = O;
}

} // namespace rlb
