// Device-side lattice tables and per-node physics for the direct-coupling LBM
// step (Astoul et al., arXiv:2004.14887).  Everything here runs in registers:
// the equilibrium (Sec. 2, Eq.(fEq_herm)), the BGK relaxation, and the Newton
// solve for the shared equilibrium at co-located nodes (Sec. 3.2,
// Eq.(system_fi), Eq.(updated_macro)).
//
// Populations are carried as s_i = f_i - E_i.  The FP64 form carries f
// itself (E = 0).  The FP32 and FP16-storage forms carry the deviation from
// the equilibrium of a uniform reference state, E_i = f0_i(1, ur) (the rest
// state w_i when ur = 0), and the velocity as du = u - ur: density and
// momentum sums then never cancel against O(1) values, and a mean flow ur
// costs no precision.
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

// Reference state of the shifted forms.
template <typename R>
struct Ref {
    R ur[3];
};

// Macroscopic state of a node in carried form.  SH: shifted form (rho0 = 1,
// E_i = f0_i(1, ur)); otherwise rho0 = 0 and du is u itself.
template <typename R>
struct Mac {
    R drho;    // rho - rho0
    R du[3];   // u - ur
    R u[3];    // ur + du
    R uu;      // |u|^2
    R q;       // |u|^2 - |ur|^2 = du.(2 ur + du)
};

template <int DIM, bool SH, typename R>
__device__ __forceinline__ Mac<R> make_mac(const Ref<R>& rf, R drho, const R du[3])
{
    Mac<R> m;
    m.drho = drho;
    m.uu = R(0);
    m.q = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m.du[a] = a < DIM ? du[a] : R(0);
        m.u[a] = SH ? rf.ur[a] + m.du[a] : m.du[a];
        m.uu += m.u[a] * m.u[a];
        if (SH) m.q += m.du[a] * (R(2) * rf.ur[a] + m.du[a]);
    }
    return m;
}

// B_i(ur + du) - B_i(ur), written in du so that nothing cancels:
//   3 dc + 4.5 dc (2 c_r + dc) - 1.5 du.(2 ur + du)   [+ 13.5 sum_{a!=g} h_ag
//   (du_a (2 ur_a + du_a) u_g + ur_a^2 du_g)],  c_r = xi.ur, dc = xi.du.
template <int DIM, int EQ, typename R>
__device__ __forceinline__ R eq_dbracket(int i, const Ref<R>& rf, const Mac<R>& m)
{
    R cr = R(0), dc = R(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        cr += R(cdir<DIM>(i, a)) * rf.ur[a];
        dc += R(cdir<DIM>(i, a)) * m.du[a];
    }
    R d = dc * (R(3) + R(4.5) * (R(2) * cr + dc)) - R(1.5) * m.q;
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
                t += (R(h3) - R(xg) / R(3)) *
                     (m.du[a] * (R(2) * rf.ur[a] + m.du[a]) * m.u[g] + rf.ur[a] * rf.ur[a] * m.du[g]);
            }
        d += R(13.5) * t;
    }
    return d;
}

// Equilibrium in the carried variable, s0_i = f0_i(rho, u) - E_i:
//   FP64 (E = 0):  w_i rho (1 + B_i(u));
//   shifted:       w_i (drho (1 + B_i(ur)) + rho (B_i(u) - B_i(ur))),
// where B_i(ur) is the same for every node (uniform registers) and the
// bracket difference is written in du, so only drho and du vary per lane.
template <int DIM, int EQ, bool SH, typename R>
__device__ __forceinline__ R eq_s(int i, const Ref<R>& rf, const Mac<R>& m)
{
    if constexpr (SH) {
        const R uur = rf.ur[0] * rf.ur[0] + rf.ur[1] * rf.ur[1] + (DIM == 3 ? rf.ur[2] * rf.ur[2] : R(0));
        const R br = eq_bracket<DIM, EQ, R>(i, rf.ur, uur);
        return R(Lat<DIM>::w[i]) * (m.drho * (R(1) + br) + (R(1) + m.drho) * eq_dbracket<DIM, EQ, R>(i, rf, m));
    } else {
        return R(Lat<DIM>::w[i]) * m.drho * (R(1) + eq_bracket<DIM, EQ, R>(i, m.u, m.uu));
    }
}

// d s0_i / d(drho, du_b) (= d f0_i / d(rho, u_b)).
template <int DIM, int EQ, bool SH, typename R>
__device__ __forceinline__ void eq_s_grad(int i, const Mac<R>& m, R g[4])
{
    const R rho = (SH ? R(1) : R(0)) + m.drho;
    const R wi = R(Lat<DIM>::w[i]);
    const R* u = m.u;
    const R cu = R(cdir<DIM>(i, 0)) * u[0] + R(cdir<DIM>(i, 1)) * u[1] +
                 (DIM == 3 ? R(cdir<DIM>(i, 2)) * u[2] : R(0));
    g[0] = wi * (R(1) + eq_bracket<DIM, EQ, R>(i, u, m.uu));
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

// Moments of the carried variable: drho = sum s, dj = sum xi s
// (sum E = rho0, sum xi E = rho0 ur).
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

// du = u - ur from the carried moments: u = (rho0 ur + dj) / rho, so
// du = (dj - drho ur) / rho (shifted) or dj / rho (rho0 = 0).
template <int DIM, bool SH, typename R>
__device__ __forceinline__ void velocity(const Ref<R>& rf, R drho, const R dj[3], R du[3])
{
    const R inv = R(1) / ((SH ? R(1) : R(0)) + drho);
#pragma unroll
    for (int a = 0; a < 3; ++a) du[a] = a < DIM ? (SH ? dj[a] - drho * rf.ur[a] : dj[a]) * inv : R(0);
}

// BGK relaxation towards f0(rho, u), in place on the carried variable.
template <int DIM, int EQ, bool SH, typename R>
__device__ __forceinline__ void bgk(R s[], const Ref<R>& rf, const Mac<R>& m, R keep /* 1 - 1/tau */)
{
#pragma unroll
    for (int i = 0; i < Lat<DIM>::Q; ++i) {
        const R e = eq_s<DIM, EQ, SH, R>(i, rf, m);
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

// Newton-Raphson for F(X) = sum_i G_i Phi_i (h_i - f0_i(X)) = 0, Phi = (1, xi)
// (Sec. 3.2, Eq.(system_fi)), in the carried variable (h and f0 are both
// shifted by E_i, which cancels in F).  Unknowns X = (drho, du); the
// Jacobian is analytic.  Start: raw moments of h.  Stop when |dX|_inf < tol.
// h_i is read through an accessor hv(i) (the interface kernels keep h in
// LDS, so only X, F and J occupy registers).  Returns the number of updates
// made, or -1 on failure.
// The equilibrium s0_i(X) and its gradient d s0_i / d(drho, du) together.
template <int DIM, int EQ, bool SH, typename R>
struct EqGrad {
    const Ref<R>& rf;
    __device__ __forceinline__ void operator()(int i, const Mac<R>& m, R& e, R g[4]) const
    {
        e = eq_s<DIM, EQ, SH, R>(i, rf, m);
        eq_s_grad<DIM, EQ, SH, R>(i, m, g);
    }
};

template <int DIM, int EQ, bool SH, typename R, typename HV, typename EG, bool ROLLED = (DIM == 3)>
__device__ __forceinline__ int newton_v(const HV& hv, uint32_t gamma_R_mask, R Rfac, const Ref<R>& rf, R tol,
                                        int maxit, R& drho, R du[3], const EG& eqg)
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
    velocity<DIM, SH, R>(rf, drho, j, du);
    for (int it = 1; it <= maxit; ++it) {
        const Mac<R> m = make_mac<DIM, SH, R>(rf, drho, du);
        R F[4] = {R(0), R(0), R(0), R(0)};
        R J[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) J[r][c] = R(0);
        // ROLLED (3-D, and the serving kernel): one direction at a time (the
        // index is uniform): unrolled, the interleaved equilibria and
        // gradients of all directions would set the register count of the
        // whole level kernel
        constexpr int UNROLL = ROLLED ? 1 : Q;
#pragma unroll UNROLL
        for (int i = 0; i < Q; ++i) {
            const R G = ((gamma_R_mask >> i) & 1u) ? Rfac : R(1);
            R e, g[4];
            eqg(i, m, e, g);
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
            du[b] += dX[1 + b];
            nrm = fmax(nrm, fabs(dX[1 + b]));
        }
        if (!(nrm == nrm)) return -1;
        if (nrm < tol) return it;
    }
    return -1;
}

}  // namespace dclbm
