// lbm_physics.hpp -- lattice, equilibrium, collision and equation of state for
// the gfx950 step of the chemical-potential multiphase LBM (arXiv 2205.09186).
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

// ---------------------------------------------------------------------------
// Velocity sets.
// D2Q9 in the order of Eq 2: rest, the four axis links at angles (i-1) pi/2,
// the four diagonals at angles (2i-9) pi/4.  D3Q19: rest, six axis links,
// twelve edge links.  Weights 4/9, 1/9, 1/36 (Eq 6) and 1/3, 1/18, 1/36.  The
// rest weight is the FP64 value that makes the rounded weights sum to exactly
// one, so collision adds no systematic mass: 4/9 and 1/3 rounded up by one ulp.
// ---------------------------------------------------------------------------
template <int LAT> struct Lat;

template <> struct Lat<0> {
    static constexpr int Q = 9, DIM = 2;
    __host__ __device__ static constexpr int ex(int i) {
        return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
    }
    __host__ __device__ static constexpr int ey(int i) {
        return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
    }
    __host__ __device__ static constexpr int ez(int) { return 0; }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 0x1.c71c71c71c71dp-2 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    // direction with e = -e_i
    __host__ __device__ static constexpr int opp(int i) {
        return i == 0 ? 0 : (i < 5 ? (i + 1) % 4 + 1 : (i - 3) % 4 + 5);
    }
};

template <> struct Lat<1> {
    static constexpr int Q = 19, DIM = 3;
    // rest; +x -x +y -y +z -z; xy edges; xz edges; yz edges
    __host__ __device__ static constexpr int ex(int i) {
        return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
             : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
    }
    __host__ __device__ static constexpr int ey(int i) {
        return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
             : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
    }
    __host__ __device__ static constexpr int ez(int i) {
        return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
             : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 0x1.5555555555556p-2 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    // direction with e = -e_i (the table pairs them as odd, even)
    __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : (i % 2 ? i + 1 : i - 1); }
};

// ---------------------------------------------------------------------------
// Collision at one node: SRT reduction of Eq 1 with exact-difference forcing
// (Eq 8), equilibrium of Eq 6 with cs^2 = 1/3:
//   f*_i = feq_i(rho, u + du) + (1 - 1/tau) (f_i - feq_i(rho, u)),  du = F/rho.
// ---------------------------------------------------------------------------
// D2Q9 moment basis of Eq 3: rows rho, e, eps, j_x, q_x, j_y, q_y, p_xx,
// p_xy; columns the directions of Eq 2.  The rows are orthogonal with squared
// norms 9, 36, 36, 6, 12, 6, 12, 4, 4, so M^-1 = M^T diag(1 / |row|^2).
__host__ __device__ constexpr int mrt_m(int k, int i)
{
    constexpr signed char T[9][9] = {
        {  1,  1,  1,  1,  1,  1,  1,  1,  1 },
        { -4, -1, -1, -1, -1,  2,  2,  2,  2 },
        {  4, -2, -2, -2, -2,  1,  1,  1,  1 },
        {  0,  1,  0, -1,  0,  1, -1, -1,  1 },
        {  0, -2,  0,  2,  0,  1, -1, -1,  1 },
        {  0,  0,  1,  0, -1,  1,  1, -1, -1 },
        {  0,  0, -2,  0,  2,  1,  1, -1, -1 },
        {  0,  1, -1,  1, -1,  0,  0,  0,  0 },
        {  0,  0,  0,  0,  0,  1, -1,  1, -1 },
    };
    return T[k][i];
}
constexpr double kMrtNorm2[9] = { 9, 36, 36, 6, 12, 6, 12, 4, 4 };

// Relaxation of Eq 1.  SRT: every rate 1/tau.  MRT (D2Q9): S of Eq 5 with
// s_1 = s_4 = s_6 = 1, s_2 = s_e, s_3 = s_eps, s_5 = s_7 = s_q,
// s_8 = s_9 = 1/tau; sd[k] = s_k / |row k|^2 folds M^-1's row scaling in.
struct Relax {
    double omo;      // 1 - 1/tau
    int mrt;         // nonzero: MRT
    double sd[9];
};

// MRT post-collision values at one D2Q9 node (Eq 1, 4, 8), given the
// equilibria at u and at u + du:
//   o = f - M^-1 S M (f - feq(rho,u)) + feq(rho,u+du) - feq(rho,u).
__device__ __forceinline__ void mrt_post(const double (&f)[9], const double (&fe)[9], const double (&fv)[9],
                                         const Relax& rx, double (&o)[9])
{
    double c[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double m = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) m += mrt_m(k, i) * (f[i] - fe[i]);
        c[k] = rx.sd[k] * m;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        double b = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) b += mrt_m(k, i) * c[k];
        o[i] = f[i] - b + (fv[i] - fe[i]);
    }
}

template <int LAT>
__device__ __forceinline__ void collide(const double (&f)[Lat<LAT>::Q], double rho,
                                        double jx, double jy, double jz,
                                        double Fx, double Fy, double Fz, const Relax& rx,
                                        double (&out)[Lat<LAT>::Q])
{
    using L = Lat<LAT>;
    const double ir = 1.0 / rho;
    const double ux = jx * ir, uy = jy * ir, uz = jz * ir;
    const double vx = ux + Fx * ir, vy = uy + Fy * ir, vz = uz + Fz * ir;
    const double uu = 1.0 - 1.5 * (ux * ux + uy * uy + uz * uz);
    const double vv = 1.0 - 1.5 * (vx * vx + vy * vy + vz * vz);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double wr = L::w(i) * rho;
        const double eu = L::ex(i) * ux + L::ey(i) * uy + L::ez(i) * uz;
        const double ev = L::ex(i) * vx + L::ey(i) * vy + L::ez(i) * vz;
        const double fe = wr * (uu + eu * (3.0 + 4.5 * eu));
        const double fv = wr * (vv + ev * (3.0 + 4.5 * ev));
        out[i] = fv + rx.omo * (f[i] - fe);
    }
    if constexpr (LAT == 0) {
        if (rx.mrt) {
            double fe[9], fv[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const double wr = L::w(i) * rho;
                const double eu = L::ex(i) * ux + L::ey(i) * uy;
                const double ev = L::ex(i) * vx + L::ey(i) * vy;
                fe[i] = wr * (uu + eu * (3.0 + 4.5 * eu));
                fv[i] = wr * (vv + ev * (3.0 + 4.5 * ev));
            }
            mrt_post(f, fe, fv, rx, out);
        }
    }
}

// ---------------------------------------------------------------------------
// Peng-Robinson bulk chemical potential psi'(rho) (Eq 15 without the gradient
// term, integration constant zero), scaled by k^2 (Eq 16), for 0 < rho < 1/b.  With x = b rho,
// g = 1 - x, A = sqrt2 - 1 + x, B = sqrt2 + 1 - x and A B = 1 + 2x - x^2:
//   psi' = RT ln(rho/g) - aa/(2 sqrt2 b) ln(A/B) + RT/g - aa rho/(A B).
// The three quotients share one division.
// ---------------------------------------------------------------------------
struct Eos {
    double k2RT;     // k^2 R T
    double k2c;      // k^2 aa / (2 sqrt2 b)
    double k2aa;     // k^2 a alpha(T)
    double b;
    double kappa;    // kappa-hat
    double mu_wall;  // mu_hat of the solid layers (wetting boundary, Appendix)
};

// Natural logarithm of a positive normal double by the classic argument
// reduction x = m 2^e, m in [1/sqrt2, sqrt2), and the odd series
//   ln m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),  s = (m - 1)/(m + 1),
// |s| <= 0.1716, summed to s^21 (the first omitted term is below 2^-59
// relative), then e ln2 added with ln2 split into a 42-bit head (e * head is
// exact) and a tail.  About a third of the instructions of the library log,
// within a few ulp of it; the chemical potential evaluates two per node.
// Domain: positive doubles; mu_bulk below guards its arguments.
__host__ __device__ __forceinline__ double log_pos(double x)
{
    int ex;
    double m = frexp(x, &ex);   // m in [0.5, 1)
    if (m < 0.70710678118654752440) { m += m; ex -= 1; }
    const double f = m - 1.0;   // exact
    const double s = f / (m + 1.0);
    const double t = s * s;
    double p = 2.0 / 21.0;
    p = fma(p, t, 2.0 / 19.0);
    p = fma(p, t, 2.0 / 17.0);
    p = fma(p, t, 2.0 / 15.0);
    p = fma(p, t, 2.0 / 13.0);
    p = fma(p, t, 2.0 / 11.0);
    p = fma(p, t, 2.0 / 9.0);
    p = fma(p, t, 2.0 / 7.0);
    p = fma(p, t, 2.0 / 5.0);
    p = fma(p, t, 2.0 / 3.0);
    const double r = fma(s * t, p, s + s);
    const double ln2_hi = 0x1.62e42fefa3800p-1, ln2_lo = 0x1.ef35793c76730p-45;
    const double de = (double)ex;
    return fma(de, ln2_hi, fma(de, ln2_lo, r));
}

__host__ __device__ __forceinline__ double mu_bulk(double rho, const Eos& e)
{
    const double s2 = 1.4142135623730951;
    const double x = e.b * rho;
    const double g = 1.0 - x, A = (s2 - 1.0) + x, B = (s2 + 1.0) - x;
    const double inv = 1.0 / (g * (A * B));
    const double inv_g = (A * B) * inv;
    const double inv_B = (g * A) * inv;
    const double inv_AB = g * inv;
    const double mu = e.k2RT * (log_pos(rho * inv_g) + inv_g) - e.k2c * log_pos(A * inv_B) - e.k2aa * rho * inv_AB;
    // both logarithms have positive arguments exactly for 0 < rho < 1/b;
    // outside (or for NaN) the potential is NaN, as with the library log, so a
    // state driven out of the EOS's range reports itself non-finite.  A
    // select, not a branch: the kernels keep one straight-line path.
    return (rho > 0.0 && g > 0.0) ? mu : __builtin_nan("");
}

}  // namespace lbm
