// lbm_kernels.hpp -- gfx950 kernels of the chemical-potential multiphase LBM
// step (arXiv 2205.09186): node-parallel reference kernels (one node per lane,
// neighbours from global memory / cache), compact line solves, reductions.
#pragma once

#include <hip/hip_runtime.h>
#include "lbm_physics.hpp"
#include "lbm_stencil.hpp"

namespace lbm {

struct Grid {
    int nx, ny, nz;
    long long N;     // nx*ny*nz
    long long nxy;   // nx*ny
    long long ps;    // element stride between population arrays (>= N)
};

__device__ __forceinline__ int wrapc(int a, int n)
{
    a += (a < 0) ? n : 0;
    a -= (a >= n) ? n : 0;
    return a;
}

__device__ __forceinline__ void coords(long long n, const Grid& g, int& x, int& y, int& z)
{
    z = (int)(n / g.nxy);
    long long r = n - (long long)z * g.nxy;
    y = (int)(r / g.nx);
    x = (int)(r - (long long)y * g.nx);
}

// Offsets of the periodic neighbours x+m, y+m, z+m for m in [-R, R].
template <int R, int DIM>
struct Nbr {
    int xo[2 * R + 1];
    long long yo[2 * R + 1], zo[2 * R + 1];
    __device__ __forceinline__ Nbr(int x, int y, int z, const Grid& g)
    {
#pragma unroll
        for (int m = -R; m <= R; ++m) {
            xo[m + R] = wrapc(x + m, g.nx);
            yo[m + R] = (long long)wrapc(y + m, g.ny) * g.nx;
            zo[m + R] = DIM == 3 ? (long long)wrapc(z + m, g.nz) * g.nxy : 0;
        }
    }
    __device__ __forceinline__ long long at(int dx, int dy, int dz) const
    {
        return zo[dz + R] + yo[dy + R] + xo[dx + R];
    }
};

// ---------------------------------------------------------------------------
// Explicit gradient and Laplacian of a field at one node.
// ---------------------------------------------------------------------------
template <int DIM, int SCH, int R>
__device__ __forceinline__ void grad_at(const double* __restrict__ f, const Nbr<R, DIM>& nb,
                                        double& gx, double& gy, double& gz)
{
    gx = gy = gz = 0.0;
    if constexpr (is_iso(SCH)) {
        constexpr int RZ = DIM == 3 ? radius(SCH) : 0;
        constexpr int RI = radius(SCH);
#pragma unroll
        for (int dz = -RZ; dz <= RZ; ++dz)
#pragma unroll
            for (int dy = -RI; dy <= RI; ++dy)
#pragma unroll
                for (int dx = -RI; dx <= RI; ++dx) {
                    const int sh = dx * dx + dy * dy + dz * dz;
                    const double w = iso_w(DIM, SCH, sh);
                    if (sh == 0 || w == 0.0) continue;
                    const double v = w * f[nb.at(dx, dy, dz)];
                    if (dx) gx += dx * v;
                    if (dy) gy += dy * v;
                    if (dz) gz += dz * v;
                }
    } else {
#pragma unroll
        for (int m = 1; m <= radius(SCH); ++m) {
            const double c = d1(SCH, m);
            gx += c * (f[nb.at(m, 0, 0)] - f[nb.at(-m, 0, 0)]);
            gy += c * (f[nb.at(0, m, 0)] - f[nb.at(0, -m, 0)]);
            if constexpr (DIM == 3) gz += c * (f[nb.at(0, 0, m)] - f[nb.at(0, 0, -m)]);
        }
    }
}

template <int DIM, int SCH, int R>
__device__ __forceinline__ double lap_at(const double* __restrict__ f, const Nbr<R, DIM>& nb)
{
    const double f0 = f[nb.at(0, 0, 0)];
    double s = 0.0;
    if constexpr (is_iso(SCH)) {
        constexpr int RZ = DIM == 3 ? radius(SCH) : 0;
        constexpr int RI = radius(SCH);
#pragma unroll
        for (int dz = -RZ; dz <= RZ; ++dz)
#pragma unroll
            for (int dy = -RI; dy <= RI; ++dy)
#pragma unroll
                for (int dx = -RI; dx <= RI; ++dx) {
                    const int sh = dx * dx + dy * dy + dz * dz;
                    const double w = iso_w(DIM, SCH, sh);
                    if (sh == 0 || w == 0.0) continue;
                    s += w * (f[nb.at(dx, dy, dz)] - f0);
                }
        return 2.0 * s;
    } else {
        s = DIM * d2(SCH, 0) * f0;
#pragma unroll
        for (int m = 1; m <= radius(SCH); ++m) {
            const double c = d2(SCH, m);
            s += c * (f[nb.at(m, 0, 0)] + f[nb.at(-m, 0, 0)]);
            s += c * (f[nb.at(0, m, 0)] + f[nb.at(0, -m, 0)]);
            if constexpr (DIM == 3) s += c * (f[nb.at(0, 0, m)] + f[nb.at(0, 0, -m)]);
        }
        return s;
    }
}

// ---------------------------------------------------------------------------
// Initial populations.  Storage S_i(x) holds the post-collision value that the
// next step pulls to x + e_i; so S_i(y) = feq_i(rho0(y + e_i), 0) makes the
// pulled state at time zero feq(rho0, 0).
// ---------------------------------------------------------------------------
template <int LAT>
__global__ void __launch_bounds__(256) k_init(const double* __restrict__ rho0, double* __restrict__ S, Grid g)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<1, L::DIM> nb(x, y, z, g);
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        S[(long long)i * g.ps + n] = L::w(i) * rho0[nb.at(L::ex(i), L::ey(i), L::ez(i))];
}

// Pull the Q populations of node n: f_i(x) = S_i(x - e_i).
template <int LAT>
__device__ __forceinline__ void pull(const double* __restrict__ S, const Grid& g, long long n,
                                     const Nbr<1, Lat<LAT>::DIM>& nb, double (&f)[Lat<LAT>::Q])
{
    using L = Lat<LAT>;
    (void)n;
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        f[i] = S[(long long)i * g.ps + nb.at(-L::ex(i), -L::ey(i), -L::ez(i))];
}

// Post-streaming populations of the stored state, f_i(x) = S_i(x - e_i).
template <int LAT>
__global__ void __launch_bounds__(256) k_pull_all(const double* __restrict__ S, double* __restrict__ out, Grid g)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<1, L::DIM> nb(x, y, z, g);
    double f[L::Q];
    pull<LAT>(S, g, n, nb, f);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) out[(long long)i * g.N + n] = f[i];
}

template <int LAT>
__global__ void __launch_bounds__(256) k_rho(const double* __restrict__ S, double* __restrict__ rho, Grid g)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<1, L::DIM> nb(x, y, z, g);
    double f[L::Q];
    pull<LAT>(S, g, n, nb, f);
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) r += f[i];
    rho[n] = r;
}

// mu_hat = k^2 psi'(rho) - kappa lap(rho) (Eq 16), explicit Laplacian.
template <int DIM, int SCH>
__global__ void __launch_bounds__(256) k_mu(const double* __restrict__ rho, double* __restrict__ mu, Grid g, Eos e)
{
    constexpr int R = radius(SCH);
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<R, DIM> nb(x, y, z, g);
    mu[n] = mu_bulk(rho[n], e) - e.kappa * lap_at<DIM, SCH, R>(rho, nb);
}

// mu_hat from a precomputed Laplacian field (compact schemes).
__global__ void __launch_bounds__(256) k_mu_lap(const double* __restrict__ rho, const double* __restrict__ lap,
                                                double* __restrict__ mu, long long N, Eos e)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    mu[n] = mu_bulk(rho[n], e) - e.kappa * lap[n];
}

// Force F = -rho grad(mu_hat) + cs^2 grad(rho) at one node (Eq 12).
template <int LAT, int SCH>
__device__ __forceinline__ void force_at(const double* __restrict__ rho_f, const double* __restrict__ mu_f,
                                         const double* __restrict__ grho, const double* __restrict__ gmu,
                                         const Grid& g, long long n, int x, int y, int z, double rho,
                                         double& Fx, double& Fy, double& Fz)
{
    using L = Lat<LAT>;
    constexpr double cs2 = 1.0 / 3.0;
    double rx, ry, rz, mx, my, mz;
    if constexpr (is_compact(SCH)) {
        rx = grho[n]; ry = grho[g.N + n]; rz = L::DIM == 3 ? grho[2 * g.N + n] : 0.0;
        mx = gmu[n]; my = gmu[g.N + n]; mz = L::DIM == 3 ? gmu[2 * g.N + n] : 0.0;
    } else {
        constexpr int R = radius(SCH);
        Nbr<R, L::DIM> nb(x, y, z, g);
        grad_at<L::DIM, SCH, R>(rho_f, nb, rx, ry, rz);
        grad_at<L::DIM, SCH, R>(mu_f, nb, mx, my, mz);
    }
    Fx = -rho * mx + cs2 * rx;
    Fy = -rho * my + cs2 * ry;
    Fz = -rho * mz + cs2 * rz;
}

// One full node update: pull, moments (Eq 7), force, collision; store locally.
template <int LAT, int SCH>
__global__ void __launch_bounds__(256) k_collide(const double* __restrict__ S, double* __restrict__ Sn,
                                                 const double* __restrict__ rho_f, const double* __restrict__ mu_f,
                                                 const double* __restrict__ grho, const double* __restrict__ gmu,
                                                 Grid g, double one_m_omega)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<1, L::DIM> nb(x, y, z, g);
    double f[L::Q], out[L::Q];
    pull<LAT>(S, g, n, nb, f);
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        r += f[i];
        jx += L::ex(i) * f[i]; jy += L::ey(i) * f[i]; jz += L::ez(i) * f[i];
    }
    double Fx, Fy, Fz;
    force_at<LAT, SCH>(rho_f, mu_f, grho, gmu, g, n, x, y, z, r, Fx, Fy, Fz);
    collide<LAT>(f, r, jx, jy, jz, Fx, Fy, Fz, one_m_omega, out);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) Sn[(long long)i * g.ps + n] = out[i];
}

// NaN-propagating maximum.
__device__ __forceinline__ double nmax(double a, double b) { return (a > b || a != a) ? a : b; }

template <int BS>
__device__ __forceinline__ void block_reduce(double& mx, double& sm)
{
    __shared__ double smx[BS / 64], ssm[BS / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = nmax(mx, __shfl_xor(mx, o));
        sm += __shfl_xor(sm, o);
    }
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
    if (ln == 0) { smx[wv] = mx; ssm[wv] = sm; }
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = smx[0]; sm = ssm[0];
        for (int k = 1; k < BS / 64; ++k) { mx = nmax(mx, smx[k]); sm += ssm[k]; }
    }
}

// Macroscopic fields and observables: rho, v = u + F/(2 rho); per-block
// (max |v|, sum rho) partials in fixed order.
template <int LAT, int SCH>
__global__ void __launch_bounds__(256) k_macros(const double* __restrict__ S,
                                                const double* __restrict__ rho_f, const double* __restrict__ mu_f,
                                                const double* __restrict__ grho, const double* __restrict__ gmu,
                                                Grid g, double* __restrict__ orho, double* __restrict__ ovx,
                                                double* __restrict__ ovy, double* __restrict__ ovz,
                                                double* __restrict__ partial)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double vmax = 0.0, msum = 0.0;
    if (n < g.N) {
        int x, y, z;
        coords(n, g, x, y, z);
        Nbr<1, L::DIM> nb(x, y, z, g);
        double f[L::Q];
        pull<LAT>(S, g, n, nb, f);
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            r += f[i];
            jx += L::ex(i) * f[i]; jy += L::ey(i) * f[i]; jz += L::ez(i) * f[i];
        }
        double Fx, Fy, Fz;
        force_at<LAT, SCH>(rho_f, mu_f, grho, gmu, g, n, x, y, z, r, Fx, Fy, Fz);
        const double ir = 1.0 / r;
        const double vx = (jx + 0.5 * Fx) * ir, vy = (jy + 0.5 * Fy) * ir, vz = (jz + 0.5 * Fz) * ir;
        if (orho) orho[n] = r;
        if (ovx) ovx[n] = vx;
        if (ovy) ovy[n] = vy;
        if (ovz) ovz[n] = vz;
        vmax = sqrt(vx * vx + vy * vy + vz * vz);
        if (!(r == r) || r - r != 0.0) vmax = r - r;   // non-finite density poisons the maximum
        msum = r;
    }
    block_reduce<256>(vmax, msum);
    if (threadIdx.x == 0) { partial[2 * blockIdx.x] = vmax; partial[2 * blockIdx.x + 1] = msum; }
}

__global__ void __launch_bounds__(1024) k_reduce_final(const double* __restrict__ partial, long long nparts,
                                                       double* __restrict__ out)
{
    double mx = 0.0, sm = 0.0;
    for (long long k = threadIdx.x; k < nparts; k += 1024) {
        mx = nmax(mx, partial[2 * k]);
        sm += partial[2 * k + 1];
    }
    block_reduce<1024>(mx, sm);
    if (threadIdx.x == 0) { out[0] = mx; out[1] = sm; }
}

// ---------------------------------------------------------------------------
// Compact derivative along one axis of a periodic field (Eq 21, beta = 0).
// The cyclic tridiagonal operator factors as
//   1 + al (S + S^-1) = (1 - zS)(1 - zS^-1) / (1 + z^2),  z = (-1 + sqrt(1 - 4 al^2)) / (2 al),
// so the derivative is (1 + z^2) times a backward first-order recursion of a
// forward first-order recursion of the right-hand side.  On a periodic line
// each recursion is an infinite geometric sum; a warm-up of K points with
// |z|^K < 1e-18 makes every value exact to rounding, for any line length.
// Work item = (line, chunk of C points).
// ---------------------------------------------------------------------------
struct LineGeom {
    int n;              // points per line
    long long sa;       // stride along the line
    int n1, n2;         // counts of the two other axes
    long long s1, s2;   // their strides
    int C, nch;         // chunk length, chunks per line
    int K;              // warm-up length
};

__device__ __forceinline__ int pmod(long long i, int n)
{
    long long r = i % n;
    return (int)(r < 0 ? r + n : r);
}

__global__ void __launch_bounds__(256) k_compact_fwd(const double* __restrict__ f, double* __restrict__ w,
                                                     LineGeom lg, Compact c, double z)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nl = (long long)lg.n1 * lg.n2;
    if (t >= nl * lg.nch) return;
    const int o1 = (int)(t % lg.n1);
    const long long rest = t / lg.n1;
    const int o2 = (int)(rest % lg.n2);
    const int ch = (int)(rest / lg.n2);
    const long long base = o1 * lg.s1 + o2 * lg.s2;
    const int start = ch * lg.C;
    const int end = min(start + lg.C, lg.n);
    const double ha = 0.5 * c.ca, hb = 0.25 * c.cb, hc = c.cc / 6.0;
    double acc = 0.0;
    for (long long i = (long long)start - lg.K; i < end; ++i) {
        const int im = pmod(i, lg.n);
        const double v = ha * (f[base + pmod(i + 1, lg.n) * lg.sa] - f[base + pmod(i - 1, lg.n) * lg.sa])
                       + hb * (f[base + pmod(i + 2, lg.n) * lg.sa] - f[base + pmod(i - 2, lg.n) * lg.sa])
                       + hc * (f[base + pmod(i + 3, lg.n) * lg.sa] - f[base + pmod(i - 3, lg.n) * lg.sa]);
        acc = v + z * acc;
        if (i >= start) w[base + im * lg.sa] = acc;
    }
}

__global__ void __launch_bounds__(256) k_compact_bwd(const double* __restrict__ w, double* __restrict__ out,
                                                     LineGeom lg, double z, double scale, int accumulate)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nl = (long long)lg.n1 * lg.n2;
    if (t >= nl * lg.nch) return;
    const int o1 = (int)(t % lg.n1);
    const long long rest = t / lg.n1;
    const int o2 = (int)(rest % lg.n2);
    const int ch = (int)(rest / lg.n2);
    const long long base = o1 * lg.s1 + o2 * lg.s2;
    const int start = ch * lg.C;
    const int end = min(start + lg.C, lg.n);
    double acc = 0.0;
    for (long long i = (long long)end - 1 + lg.K; i >= start; --i) {
        const int im = pmod(i, lg.n);
        acc = w[base + im * lg.sa] + z * acc;
        if (i < end) {
            const long long o = base + im * lg.sa;
            out[o] = accumulate ? out[o] + scale * acc : scale * acc;
        }
    }
}

}  // namespace lbm
