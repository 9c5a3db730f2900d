// Device-side lattice tables and per-node physics for the direct-coupling LBM
// step (Astoul et al., arXiv:2004.14887).  Everything here runs in registers:
// the equilibrium (Sec. 2, Eq.(fEq_herm)), the BGK relaxation, and the Newton
// solve for the shared equilibrium at co-located nodes (Sec. 3.2,
// Eq.(system_fi), Eq.(updated_macro)).
//
// Populations are carried as s_i = f_i - rho0 * w_i.  The FP64 form uses
// rho0 = 0 (s = f); the FP32 and FP16-storage forms use rho0 = 1, i.e. the
// deviation from the rest state, so density and momentum sums never cancel
// against the O(1) rest weights.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dclbm {

template <int DIM>
struct Lat;

// D2Q9, numbered as the direction labels of the paper's Fig. 1:
// 0 rest, 1 E, 2 NE, 3 N, 4 NW, 5 W, 6 SW, 7 S, 8 SE.
template <>
struct Lat<2> {
    static constexpr int D = 2;
    static constexpr int Q = 9;
    static constexpr int cx[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
    static constexpr int cy[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36,
                                    1.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36};
};

// D3Q19 (Sec. 2, Eq.(xi_i), Eq.(w_i)); within each group: +x,-x,+y,-y,+z,-z,
// then the xy, xz and yz diagonals as (+,+),(-,-),(+,-),(-,+).
template <>
struct Lat<3> {
    static constexpr int D = 3;
    static constexpr int Q = 19;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

template <int DIM>
__host__ __device__ constexpr int cdir(int i, int a)
{
    return a == 0 ? Lat<DIM>::cx[i] : (a == 1 ? Lat<DIM>::cy[i] : Lat<DIM>::cz[i]);
}

// Equilibrium bracket B_i(u) = xi.u/c^2 + ((xi.u)^2 - c^2 u.u)/(2c^4)
//                              [+ sum_{a!=g} (xi_a^2 xi_g - c^2 xi_g) u_a^2 u_g / (2 c^6)]
// so that f0_i = w_i rho (1 + B_i).  c^2 = 1/3.
template <int DIM, int EQ, typename R>
__device__ __forceinline__ R eq_bracket(int i, const R u[3], R uu)
{
    const R cu = R(cdir<DIM>(i, 0)) * u[0] + R(cdir<DIM>(i, 1)) * u[1] +
                 (DIM == 3 ? R(cdir<DIM>(i, 2)) * u[2] : R(0));
    R b = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
    if constexpr (EQ == 3) {
        R t = R(0);
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int g = 0; g < DIM; ++g) {
                if (a == g) continue;
                const int h3 = cdir<DIM>(i, a) * cdir<DIM>(i, a) * cdir<DIM>(i, g);
                const int xg = cdir<DIM>(i, g);
                if (h3 == 0 && xg == 0) continue;
                t += (R(h3) - R(xg) / R(3)) * u[a] * u[a] * u[g];
            }
        b += R(13.5) * t;   // 1/(2 c^6) = 27/2
    }
    return b;
}

// Equilibrium in the carried variable: s0_i = f0_i - rho0 w_i
//   = w_i (drho + rho B_i),  with rho = rho0 + drho.
template <int DIM, int EQ, typename R>
__device__ __forceinline__ R eq_s(int i, R rho0, R drho, const R u[3], R uu)
{
    const R rho = rho0 + drho;
    return R(Lat<DIM>::w[i]) * (drho + rho * eq_bracket<DIM, EQ, R>(i, u, uu));
}

// d s0_i / d(drho, u_b)
template <int DIM, int EQ, typename R>
__device__ __forceinline__ void eq_s_grad(int i, R rho0, R drho, const R u[3], R uu, R g[4])
{
    const R rho = rho0 + drho;
    const R wi = R(Lat<DIM>::w[i]);
    const R cu = R(cdir<DIM>(i, 0)) * u[0] + R(cdir<DIM>(i, 1)) * u[1] +
                 (DIM == 3 ? R(cdir<DIM>(i, 2)) * u[2] : R(0));
    g[0] = wi * (R(1) + eq_bracket<DIM, EQ, R>(i, u, uu));
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const R xb = R(cdir<DIM>(i, b));
        R v = R(3) * xb + R(9) * cu * xb - R(3) * u[b];
        if constexpr (EQ == 3) {
            R t = R(0);
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int gg = 0; gg < DIM; ++gg) {
                    if (a == gg) continue;
                    const R h3 = R(cdir<DIM>(i, a) * cdir<DIM>(i, a) * cdir<DIM>(i, gg)) -
                                 R(cdir<DIM>(i, gg)) / R(3);
                    R dd = R(0);
                    if (a == b) dd += R(2) * u[a] * u[gg];
                    if (gg == b) dd += u[a] * u[a];
                    t += h3 * dd;
                }
            v += R(13.5) * t;
        }
        g[1 + b] = wi * rho * v;
    }
    if (DIM == 2) g[3] = R(0);
}

// Moments of the carried variable: drho = sum s, j = sum xi s  (sum w = 1, sum w xi = 0).
template <int DIM, typename R>
__device__ __forceinline__ void moments(const R s[], R& drho, R j[3])
{
    drho = R(0);
    j[0] = j[1] = j[2] = R(0);
#pragma unroll
    for (int i = 0; i < Lat<DIM>::Q; ++i) {
        drho += s[i];
        if (cdir<DIM>(i, 0)) j[0] += R(cdir<DIM>(i, 0)) * s[i];
        if (cdir<DIM>(i, 1)) j[1] += R(cdir<DIM>(i, 1)) * s[i];
        if (DIM == 3 && cdir<DIM>(i, 2)) j[2] += R(cdir<DIM>(i, 2)) * s[i];
    }
}

// BGK relaxation towards f0(rho, u), in place on the carried variable.
template <int DIM, int EQ, typename R>
__device__ __forceinline__ void bgk(R s[], R rho0, R drho, const R u[3], R keep /* 1 - 1/tau */)
{
    const R uu = u[0] * u[0] + u[1] * u[1] + (DIM == 3 ? u[2] * u[2] : R(0));
#pragma unroll
    for (int i = 0; i < Lat<DIM>::Q; ++i) {
        const R e = eq_s<DIM, EQ, R>(i, rho0, drho, u, uu);
        s[i] = e + keep * (s[i] - e);
    }
}

// Gaussian elimination with partial pivoting, n = DIM + 1 <= 4, in registers.
template <int N, typename R>
__device__ __forceinline__ bool solve_small(R A[4][4], R b[4], R x[4])
{
#pragma unroll
    for (int k = 0; k < N; ++k) {
        int p = k;
        R best = fabs(A[k][k]);
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const R v = fabs(A[r][k]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (!(best > R(0))) return false;
        if (p != k) {
#pragma unroll
            for (int r = k + 1; r < N; ++r) {
                if (r != p) continue;
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    const R t = A[k][c];
                    A[k][c] = A[r][c];
                    A[r][c] = t;
                }
                const R t = b[k];
                b[k] = b[r];
                b[r] = t;
            }
        }
        const R inv = R(1) / A[k][k];
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const R m = A[r][k] * inv;
#pragma unroll
            for (int c = k; c < N; ++c) A[r][c] -= m * A[k][c];
            b[r] -= m * b[k];
        }
    }
#pragma unroll
    for (int r = N - 1; r >= 0; --r) {
        R s = b[r];
#pragma unroll
        for (int c = r + 1; c < N; ++c) s -= A[r][c] * x[c];
        x[r] = s / A[r][r];
    }
    return true;
}

// Newton-Raphson for F(X) = sum_i G_i Phi_i (h_i - f0_i(X)) = 0, Phi = (1, xi),
// in the carried variable (h and f0 both shifted by rho0 w_i, which cancels
// in F because sum_i G_i Phi_i w_i is common to both terms).  Unknowns
// (drho, u).  Start: raw moments of h.  Stop when |dX|_inf < tol.
// Returns the number of updates made, or -1 on failure.
template <int DIM, int EQ, typename R>
__device__ __forceinline__ int newton(const R h[], uint32_t gamma_R_mask, R Rfac, R rho0, R tol,
                                      int maxit, R& drho, R u[3])
{
    constexpr int Q = Lat<DIM>::Q;
    constexpr int N = DIM + 1;
    R j[3];
    moments<DIM, R>(h, drho, j);
    const R rho_init = rho0 + drho;
    u[0] = j[0] / rho_init;
    u[1] = j[1] / rho_init;
    u[2] = DIM == 3 ? j[2] / rho_init : R(0);
    for (int it = 1; it <= maxit; ++it) {
        const R uu = u[0] * u[0] + u[1] * u[1] + (DIM == 3 ? u[2] * u[2] : R(0));
        R F[4] = {R(0), R(0), R(0), R(0)};
        R J[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) J[r][c] = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R G = ((gamma_R_mask >> i) & 1u) ? Rfac : R(1);
            const R e = eq_s<DIM, EQ, R>(i, rho0, drho, u, uu);
            R g[4];
            eq_s_grad<DIM, EQ, R>(i, rho0, drho, u, uu, g);
            const R d = G * (h[i] - e);
            const R phi[4] = {R(1), R(cdir<DIM>(i, 0)), R(cdir<DIM>(i, 1)), R(cdir<DIM>(i, 2))};
#pragma unroll
            for (int r = 0; r < N; ++r) {
                if (phi[r] == R(0)) continue;
                F[r] += phi[r] * d;
#pragma unroll
                for (int c = 0; c < N; ++c) J[r][c] -= G * phi[r] * g[c];
            }
        }
        R rhs[4] = {-F[0], -F[1], -F[2], -F[3]};
        R dX[4] = {R(0), R(0), R(0), R(0)};
        if (!solve_small<N, R>(J, rhs, dX)) return -1;
        drho += dX[0];
        R nrm = fabs(dX[0]);
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            u[b] += dX[1 + b];
            nrm = fmax(nrm, fabs(dX[1 + b]));
        }
        if (!(nrm == nrm)) return -1;
        if (nrm < tol) return it;
    }
    return -1;
}

// The same Newton iteration with h_i read through an accessor hv(i) (the
// interface kernels keep h in LDS, so only X, F and J occupy registers).
template <int DIM, int EQ, typename R, typename HV>
__device__ __forceinline__ int newton_v(const HV& hv, uint32_t gamma_R_mask, R Rfac, R rho0, R tol, int maxit,
                                        R& drho, R u[3])
{
    constexpr int Q = Lat<DIM>::Q;
    constexpr int N = DIM + 1;
    R j[3] = {R(0), R(0), R(0)};
    drho = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R v = hv(i);
        drho += v;
        if (cdir<DIM>(i, 0)) j[0] += R(cdir<DIM>(i, 0)) * v;
        if (cdir<DIM>(i, 1)) j[1] += R(cdir<DIM>(i, 1)) * v;
        if (DIM == 3 && cdir<DIM>(i, 2)) j[2] += R(cdir<DIM>(i, 2)) * v;
    }
    const R rho_init = rho0 + drho;
    u[0] = j[0] / rho_init;
    u[1] = j[1] / rho_init;
    u[2] = DIM == 3 ? j[2] / rho_init : R(0);
    for (int it = 1; it <= maxit; ++it) {
        const R uu = u[0] * u[0] + u[1] * u[1] + (DIM == 3 ? u[2] * u[2] : R(0));
        R F[4] = {R(0), R(0), R(0), R(0)};
        R J[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) J[r][c] = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R G = ((gamma_R_mask >> i) & 1u) ? Rfac : R(1);
            const R e = eq_s<DIM, EQ, R>(i, rho0, drho, u, uu);
            R g[4];
            eq_s_grad<DIM, EQ, R>(i, rho0, drho, u, uu, g);
            const R d = G * (hv(i) - e);
            const R phi[4] = {R(1), R(cdir<DIM>(i, 0)), R(cdir<DIM>(i, 1)), R(cdir<DIM>(i, 2))};
#pragma unroll
            for (int r = 0; r < N; ++r) {
                if (phi[r] == R(0)) continue;
                F[r] += phi[r] * d;
#pragma unroll
                for (int c = 0; c < N; ++c) J[r][c] -= G * phi[r] * g[c];
            }
        }
        R rhs[4] = {-F[0], -F[1], -F[2], -F[3]};
        R dX[4] = {R(0), R(0), R(0), R(0)};
        if (!solve_small<N, R>(J, rhs, dX)) return -1;
        drho += dX[0];
        R nrm = fabs(dX[0]);
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            u[b] += dX[1 + b];
            nrm = fmax(nrm, fabs(dX[1 + b]));
        }
        if (!(nrm == nrm)) return -1;
        if (nrm < tol) return it;
    }
    return -1;
}

}  // namespace dclbm
