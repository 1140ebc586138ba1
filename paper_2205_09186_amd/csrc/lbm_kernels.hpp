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
    // wetting boundary (Appendix): per node 0 = fluid, l = 1..r the solid
    // layer, kDeepSolid beyond the last layer; nullptr = no solid nodes
    const unsigned char* wl;
};

constexpr unsigned char kDeepSolid = 255;

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
//   With solid nodes a value that the next step sends into the solid comes
// back to its own node reversed (halfway bounce-back), so there it carries
// rho0 of the node itself; solid nodes hold zeros, which nothing reads.
template <int LAT>
__global__ void __launch_bounds__(256) k_init(const double* __restrict__ rho0, double* __restrict__ S, Grid g)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<1, L::DIM> nb(x, y, z, g);
    if (g.wl && g.wl[n] != 0) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) S[(long long)i * g.ps + n] = 0.0;
        return;
    }
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const long long m = nb.at(L::ex(i), L::ey(i), L::ez(i));
        S[(long long)i * g.ps + n] = L::w(i) * rho0[(g.wl && g.wl[m] != 0) ? n : m];
    }
}

// Pull the Q populations of fluid node n: f_i(x) = S_i(x - e_i), or, when
// x - e_i is solid, the node's own post-collision value in the opposite
// direction, S_opp(i)(x) (halfway bounce-back at the wetting boundary).
template <int LAT>
__device__ __forceinline__ void pull(const double* __restrict__ S, const Grid& g, long long n,
                                     const Nbr<1, Lat<LAT>::DIM>& nb, double (&f)[Lat<LAT>::Q])
{
    using L = Lat<LAT>;
    if (g.wl) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const long long m = nb.at(-L::ex(i), -L::ey(i), -L::ez(i));
            f[i] = g.wl[m] != 0 ? S[(long long)L::opp(i) * g.ps + n] : S[(long long)i * g.ps + m];
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        f[i] = S[(long long)i * g.ps + nb.at(-L::ex(i), -L::ey(i), -L::ez(i))];
}

// ---------------------------------------------------------------------------
// Wetting boundary (Appendix).  The solid layers are counted through the
// lattice directions: a solid node joins layer l when a neighbour x + e_i is
// in layer l - 1 (layer 0 = fluid), for l = 1..r, r the radius of the central
// scheme.  Their density is Eq A.1, the lattice-weighted mean over the
// neighbours in layer l - 1; their chemical potential is the given mu_wall.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wall_mark(unsigned char* __restrict__ wl, long long N)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) wl[n] = wl[n] != 0 ? kDeepSolid : 0;
}

// Nodes still unassigned that touch layer l - 1 join layer l.  Concurrent
// writes only turn kDeepSolid into l, never into l - 1, so the test is exact.
template <int LAT>
__global__ void __launch_bounds__(256) k_wall_layer(unsigned char* __restrict__ wl, Grid g, int l)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N || wl[n] != kDeepSolid) return;
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<1, L::DIM> nb(x, y, z, g);
    bool touch = false;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) touch |= wl[nb.at(L::ex(i), L::ey(i), L::ez(i))] == l - 1;
    if (touch) wl[n] = (unsigned char)l;
}

// Per-node mask for the fast path's bounce-back: bit 31 marks a solid node;
// on a fluid node bit i marks a solid source x - e_i.
template <int LAT>
__global__ void __launch_bounds__(256) k_wall_bits(const unsigned char* __restrict__ wl, unsigned* __restrict__ wb,
                                                   Grid g)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    if (wl[n] != 0) { wb[n] = 1u << 31; return; }
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<1, L::DIM> nb(x, y, z, g);
    unsigned m = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i)
        if (wl[nb.at(-L::ex(i), -L::ey(i), -L::ez(i))] != 0) m |= 1u << i;
    wb[n] = m;
}

// Eq A.1 on layer l; the l = 1 launch also gives the solid beyond the last
// layer a harmless density of 1 (no fluid stencil reaches it).
template <int LAT>
__global__ void __launch_bounds__(256) k_wall_rho(double* __restrict__ rho, Grid g, int l)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int ln = g.wl[n];
    if (ln == kDeepSolid) {
        if (l == 1) rho[n] = 1.0;
        return;
    }
    if (ln != l) return;
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<1, L::DIM> nb(x, y, z, g);
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const long long m = nb.at(L::ex(i), L::ey(i), L::ez(i));
        if (g.wl[m] == l - 1) { num += L::w(i) * rho[m]; den += L::w(i); }
    }
    rho[n] = num / den;
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
    if (g.wl && g.wl[n] != 0) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) f[i] = 0.0;
    } else {
        pull<LAT>(S, g, n, nb, f);
    }
#pragma unroll
    for (int i = 0; i < L::Q; ++i) out[(long long)i * g.N + n] = f[i];
}

template <int LAT>
__global__ void __launch_bounds__(256) k_rho(const double* __restrict__ S, double* __restrict__ rho, Grid g)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N || (g.wl && g.wl[n] != 0)) return;   // solid: k_wall_rho
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
    if (g.wl && g.wl[n] != 0) {      // the wall's chemical potential
        mu[n] = e.mu_wall;
        return;
    }
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<R, DIM> nb(x, y, z, g);
    mu[n] = mu_bulk(rho[n], e) - e.kappa * lap_at<DIM, SCH, R>(rho, nb);
}

// mu_hat = k^2 psi'(rho) - kappa (lap_x + lap_y [+ lap_z]) (Eq 16) from the
// per-axis terms of a compact Laplacian, summed in axis order.
__global__ void __launch_bounds__(256) k_mu_sum(const double* __restrict__ rho, const double* __restrict__ lap,
                                                int dim, long long N, Eos e, double* __restrict__ mu)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double l = lap[n] + lap[N + n];
    if (dim == 3) l += lap[2 * N + n];
    mu[n] = mu_bulk(rho[n], e) - e.kappa * l;
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
                                                 Grid g, Relax rx)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N || (g.wl && g.wl[n] != 0)) return;   // no collision in the solid
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
    collide<LAT>(f, r, jx, jy, jz, Fx, Fy, Fz, rx, out);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) Sn[(long long)i * g.ps + n] = out[i];
}

// Force (Eq 12) at every node from rho, mu_hat and, for the compact schemes,
// the precomputed gradient fields; F stored as DIM planes of N.
template <int LAT, int SCH>
__global__ void __launch_bounds__(256) k_force_node(const double* __restrict__ rho, const double* __restrict__ mu,
                                                    const double* __restrict__ grho, const double* __restrict__ gmu,
                                                    Grid g, double* __restrict__ F)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    coords(n, g, x, y, z);
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    if (!(g.wl && g.wl[n] != 0)) force_at<LAT, SCH>(rho, mu, grho, gmu, g, n, x, y, z, rho[n], Fx, Fy, Fz);
    F[n] = Fx;
    F[g.N + n] = Fy;
    if constexpr (Lat<LAT>::DIM == 3) F[2 * g.N + n] = Fz;
}

// Gradient and Laplacian of a field with an explicit or isotropic scheme.
template <int DIM, int SCH>
__global__ void __launch_bounds__(256) k_gradlap(const double* __restrict__ in, double* __restrict__ grad,
                                                 double* __restrict__ lap, Grid g)
{
    constexpr int R = radius(SCH);
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    coords(n, g, x, y, z);
    Nbr<R, DIM> nb(x, y, z, g);
    double gx, gy, gz;
    grad_at<DIM, SCH, R>(in, nb, gx, gy, gz);
    grad[n] = gx;
    grad[g.N + n] = gy;
    if constexpr (DIM == 3) grad[2 * g.N + n] = gz;
    if (lap) lap[n] = lap_at<DIM, SCH, R>(in, nb);
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
    if (n < g.N && g.wl && g.wl[n] != 0) {    // solid: no fluid there
        if (orho) orho[n] = 0.0;
        if (ovx) ovx[n] = 0.0;
        if (ovy) ovy[n] = 0.0;
        if (ovz) ovz[n] = 0.0;
    } else if (n < g.N) {
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

// Nodes whose initial density lies outside (0, rmax) (NaN included), solid
// nodes (wl != 0) skipped: per-block counts in the sum slot of the partials.
__global__ void __launch_bounds__(256) k_check_rho(const double* __restrict__ rho,
                                                   const unsigned char* __restrict__ wl, long long N, double rmax,
                                                   double* __restrict__ partial)
{
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    double mx = 0.0, bad = 0.0;
    if (n < N && !(wl && wl[n])) {
        const double r = rho[n];
        bad = (r > 0.0 && r < rmax) ? 0.0 : 1.0;
    }
    block_reduce<256>(mx, bad);
    if (threadIdx.x == 0) { partial[2 * blockIdx.x] = 0.0; partial[2 * blockIdx.x + 1] = bad; }
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

// Forward recursion w_i = v_i + z w_{i-1} along lines of a non-unit-stride
// axis, v_i the right-hand side of Eq 21.  One thread per (line, chunk of C);
// the recursion starts K points early, where |z|^K < 1e-18.  Lanes run along x,
// so every load is coalesced; a seven-point register window leaves one new
// load per point.
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
    const int n = lg.n;
    const long long sa = lg.sa;
    const int start = ch * lg.C;
    const int end = min(start + lg.C, n);
    const double ha = 0.5 * c.ca, hb = 0.25 * c.cb, hc = c.cc / 6.0;
    const int i0 = start - lg.K;
    double r[7];   // f at i-3 .. i+3
#pragma unroll
    for (int k = 0; k < 7; ++k) r[k] = f[base + pmod((long long)i0 - 3 + k, n) * sa];
    int jn = pmod((long long)i0 + 4, n);   // next point entering the window
    int im = pmod(i0, n);                  // current point
    double acc = 0.0;
#pragma unroll 8
    for (int i = i0; i < end; ++i) {
        const double v = ha * (r[4] - r[2]) + hb * (r[5] - r[1]) + hc * (r[6] - r[0]);
        acc = v + z * acc;
        if (i >= start) w[base + im * sa] = acc;
#pragma unroll
        for (int k = 0; k < 6; ++k) r[k] = r[k + 1];
        r[6] = f[base + jn * sa];
        jn = jn + 1 == n ? 0 : jn + 1;
        im = im + 1 == n ? 0 : im + 1;
    }
}

// What the last pass of a compact derivative D g writes at node o.
enum CompactOut { C_STORE = 0, C_ADD = 1, C_FORCE = 2, C_MU = 3 };
struct CompactSink {
    double* out;
    int mode;             // C_STORE: out = D g; C_ADD: out += D g;
    const double* rho;    // C_FORCE: out = -rho D mu_hat + cs^2 G[rho] (Eq 12), g = mu_hat,
    const double* grad;   //          grad = the same component of G[rho];
    Eos eos;              // C_MU: the last term of the Laplacian, out = mu_hat =
                          //       k^2 psi'(rho) - kappa (grad + D g) (Eq 16), grad = the
                          //       sum of the other axes' terms
    __device__ __forceinline__ void put(long long o, double d) const
    {
        if (mode == C_FORCE) out[o] = -rho[o] * d + (1.0 / 3.0) * grad[o];
        else if (mode == C_ADD) out[o] += d;
        else if (mode == C_MU) out[o] = mu_bulk(rho[o], eos) - eos.kappa * (grad[o] + d);
        else out[o] = d;
    }
};

// The sink of a run of M points (element offsets o, values v, ok = written):
// every load of the run is issued before its first store, so the run costs
// one memory round trip rather than one per point.
template <int M, typename T>
__device__ __forceinline__ void sink_run_impl(int mode, const Eos& eos, double* __restrict__ out,
                                              const double* __restrict__ rho, const double* __restrict__ gr,
                                              const T (&o)[M], const double (&v)[M], const bool (&ok)[M])
{
    if (mode == C_STORE) {
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (ok[m]) out[o[m]] = v[m];
        return;
    }
    double a[M], b[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        a[m] = ok[m] ? (mode == C_ADD ? out[o[m]] : rho[o[m]]) : 1.0;
        b[m] = ok[m] && mode != C_ADD ? gr[o[m]] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (!ok[m]) continue;
        if (mode == C_ADD) out[o[m]] = a[m] + v[m];
        else if (mode == C_FORCE) out[o[m]] = -a[m] * v[m] + (1.0 / 3.0) * b[m];
        else out[o[m]] = mu_bulk(a[m], eos) - eos.kappa * (b[m] + v[m]);
    }
}

template <int M, typename T>
__device__ __forceinline__ void sink_run(const CompactSink& k, const T (&o)[M], const double (&v)[M],
                                         const bool (&ok)[M])
{
    sink_run_impl<M, T>(k.mode, k.eos, k.out, k.rho, k.grad, o, v, ok);
}

// Backward recursion y_i = w_i + z y_{i+1}; the sink receives scale * y.
__global__ void __launch_bounds__(256) k_compact_bwd(const double* __restrict__ w, CompactSink sink,
                                                     LineGeom lg, double z, double scale)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nl = (long long)lg.n1 * lg.n2;
    if (t >= nl * lg.nch) return;
    const int o1 = (int)(t % lg.n1);
    const long long rest = t / lg.n1;
    const int o2 = (int)(rest % lg.n2);
    const int ch = (int)(rest / lg.n2);
    const long long base = o1 * lg.s1 + o2 * lg.s2;
    const int n = lg.n;
    const long long sa = lg.sa;
    const int start = ch * lg.C;
    const int end = min(start + lg.C, n);
    const int i0 = end - 1 + lg.K;
    int im = pmod(i0, n);
    double acc = 0.0;
    // warm-up (nothing is written), then the chunk in runs of 16 points whose
    // sink loads are all issued before the run's stores
#pragma unroll 8
    for (int i = i0; i >= end; --i) {
        acc = w[base + im * sa] + z * acc;
        im = im == 0 ? n - 1 : im - 1;
    }
    for (int i = end - 1; i >= start; i -= 16) {
        long long o[16];
        double v[16];
        bool ok[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            ok[m] = i - m >= start;
            o[m] = base + im * sa;
            acc = ok[m] ? w[o[m]] + z * acc : acc;
            v[m] = scale * acc;
            im = im == 0 ? n - 1 : im - 1;
        }
        sink_run<16, long long>(sink, o, v, ok);
    }
}

// Compact derivative (Eq 21) of f along one periodic line of n <= 64 kLineSeg
// points, by one wavefront: lane l takes the segment [l L, l L + L_l) of the
// line (L = ceil(n / 64)).  Both recursions of the factorised cyclic solve
// (a_i = v_i + z a_{i-1}, then y_i = a_i + z y_{i+1}, times scale = 1 + z^2)
// run in registers from a zero start; the true value entering each segment
// follows from a scan over the lanes of the pairs (z^L_l, local end), closed
// around the periodic line by 1 / (1 - z^n).  Exact, no warm-up.  The lane's
// results land in y[0 .. Ll) for the points s0 .. s0 + Ll - 1.  The field
// value at offset o comes from ld(o).
constexpr int kLineSeg = 16;   // lines of up to 64 * 16 = 1024 nodes

template <class Load>
__device__ __forceinline__ void wave_line(Load&& ld, long long base, long long sa, int n, int lane, const Compact& c,
                                          double z, double scale, double (&y)[kLineSeg], int& s0, int& Ll)
{
    const double ha = 0.5 * c.ca, hb = 0.25 * c.cb, hc = c.cc / 6.0;
    const int L = (n + 63) / 64;
    s0 = min(lane * L, n);
    Ll = min(L, n - s0);
    double r[kLineSeg + 6];
#pragma unroll
    for (int k = 0; k < kLineSeg + 6; ++k) {
        int idx = s0 - 3 + k;               // in [-3, n + 2]; n >= 4
        idx += idx < 0 ? n : 0;
        idx -= idx >= n ? n : 0;
        r[k] = k < Ll + 6 ? ld(base + idx * sa) : 0.0;
    }
    double acc = 0.0, pz = 1.0;
#pragma unroll
    for (int i = 0; i < kLineSeg; ++i) {
        if (i < Ll) {
            acc = ha * (r[i + 4] - r[i + 2]) + hb * (r[i + 5] - r[i + 1]) + hc * (r[i + 6] - r[i]) + z * acc;
            r[i] = acc;
            pz *= z;
        }
    }
    // forward: T_l = E_l + z^L_l T_{l-1}, cyclic over the lanes
    double P = pz, V = acc;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const double Pp = __shfl_up(P, s, 64), Vp = __shfl_up(V, s, 64);
        if (lane >= s) { V += P * Vp; P *= Pp; }
    }
    const double Tlast = __shfl(V, 63, 64) / (1.0 - __shfl(P, 63, 64));
    double cin = __shfl_up(V + P * Tlast, 1, 64);
    if (lane == 0) cin = Tlast;
    double q = z;
#pragma unroll
    for (int i = 0; i < kLineSeg; ++i)
        if (i < Ll) { r[i] += q * cin; q *= z; }
    acc = 0.0;
#pragma unroll
    for (int i = kLineSeg - 1; i >= 0; --i)
        if (i < Ll) { acc = r[i] + z * acc; r[i] = acc; }
    // backward: U_l = B_l + z^L_l U_{l+1}, cyclic over the lanes
    P = pz; V = acc;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const double Pn = __shfl_down(P, s, 64), Vn = __shfl_down(V, s, 64);
        if (lane + s < 64) { V += P * Vn; P *= Pn; }
    }
    const double Ufirst = __shfl(V, 0, 64) / (1.0 - __shfl(P, 0, 64));
    double cr = __shfl_down(V + P * Ufirst, 1, 64);
    if (lane == 63) cr = Ufirst;
    q = z;
#pragma unroll
    for (int i = kLineSeg - 1; i >= 0; --i) {
        y[i] = 0.0;
        if (i < Ll) { y[i] = scale * (r[i] + q * cr); q *= z; }
    }
}

// Compact derivative of lines of up to 1024 points, one wavefront per line
// (wave_line), into the sink.
__global__ void __launch_bounds__(256) k_compact_wave(const double* __restrict__ f, CompactSink sink, LineGeom lg,
                                                      Compact c, double z, double scale)
{
    const int lane = threadIdx.x & 63;
    const long long t = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= (long long)lg.n1 * lg.n2) return;     // whole wavefront leaves
    const long long base = (t % lg.n1) * lg.s1 + (t / lg.n1) * lg.s2;
    double y[kLineSeg];
    int s0, Ll;
    wave_line([&](long long o) { return f[o]; }, base, lg.sa, lg.n, lane, c, z, scale, y, s0, Ll);
    long long o[kLineSeg];
    bool ok[kLineSeg];
#pragma unroll
    for (int i = 0; i < kLineSeg; ++i) {
        ok[i] = i < Ll;
        o[i] = base + (ok[i] ? s0 + i : 0) * lg.sa;
    }
    sink_run<kLineSeg, long long>(sink, o, y, ok);
}

// Compact derivative along y or z of whole lines in one pass (lines of at
// most kSegMaxWavesLong * kSegLen = 384 points; lanes along x with unit stride).  A workgroup
// takes 64 neighbouring lines; wave w solves points [w S, w S + L_w) of each
// in registers.  Both recursions run locally from a zero start and are then
// made exact for the periodic line by the carries of the other segments:
//   forward   a_i = v_i + z a_{i-1}: segment w ends at E_w locally; the true
//             end T_m = sum_j z^(distance from end_j to end_m) E_j / (1 - z^n),
//             and A_i = a_i + z^(i - s_w + 1) T_{w-1};
//   backward  y_i = A_i + z y_{i+1}: segment w starts at B_w locally; the true
//             start U_m from the B_j the same way, and y_i = b_i +
//             z^(s_w + L_w - i) U_{w+1}.
// The sink receives scale * y.  Each point of g is read once (plus the
// three-point halos of the right-hand side) and each output written once.
constexpr int kSegMaxWaves = 8;
constexpr int kSegLen = 32;   // 64-point segments spill registers
constexpr int kSegMaxWavesLong = 12;   // y and z lines of up to 384 points

template <int S, int MAXW>
__global__ void __launch_bounds__(64 * MAXW)
k_compact_seg(const double* __restrict__ f, CompactSink sink, LineGeom lg, Compact c, double z, double scale,
              double zS, double zLast, double zN)
{
    __shared__ double ends[MAXW][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int W = blockDim.x >> 6;
    const int n = lg.n;
    const int groups = (lg.n1 + 63) / 64;
    const int o1 = min((int)(blockIdx.x % groups) * 64 + lane, lg.n1 - 1);
    const bool active = (int)(blockIdx.x % groups) * 64 + lane < lg.n1;
    const int o2 = (int)(blockIdx.x / groups);
    // element offsets fit 32 bits (the host launches this for N < 2^29), so
    // each load address is one register over the uniform base pointer
    const unsigned base = (unsigned)(o1 * lg.s1 + (long long)o2 * lg.s2);
    const unsigned sa = (unsigned)lg.sa;
    const char* fb = reinterpret_cast<const char*>(f);
    const int s0 = w * S;
    const int L = min(S, n - s0);
    const double ha = 0.5 * c.ca, hb = 0.25 * c.cb, hc = c.cc / 6.0;
    // g at s0 - 3 .. s0 + L + 2; the forward results replace it in place
    double r[S + 6];
#pragma unroll
    for (int k = 0; k < S + 6; ++k) {
        int idx = s0 - 3 + k;            // in [-3, n + 2]; n >= 4
        idx += idx < 0 ? n : 0;
        idx -= idx >= n ? n : 0;
        r[k] = k < L + 6 ? *reinterpret_cast<const double*>(fb + (size_t)((base + (unsigned)idx * sa) * 8u)) : 0.0;
    }
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        if (i < L) {
            const double v = ha * (r[i + 4] - r[i + 2]) + hb * (r[i + 5] - r[i + 1]) + hc * (r[i + 6] - r[i]);
            acc = v + z * acc;
            r[i] = acc;
        }
    }
    ends[w][lane] = acc;
    __syncthreads();
    {
        // true end of the previous segment (periodic), from every segment's local end
        const int m = w == 0 ? W - 1 : w - 1;
        double t = 0.0, p = 1.0;
        for (int k = 0, j = m; k < W; ++k) {
            t += p * ends[j][lane];
            p *= j == W - 1 ? zLast : zS;
            j = j == 0 ? W - 1 : j - 1;
        }
        t /= 1.0 - zN;
        double q = z;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (i < L) { r[i] += q * t; q *= z; }
        }
    }
    __syncthreads();   // every wave has read the forward ends
    acc = 0.0;
#pragma unroll
    for (int i = S - 1; i >= 0; --i) {
        if (i < L) { acc = r[i] + z * acc; r[i] = acc; }
    }
    ends[w][lane] = acc;
    __syncthreads();
    {
        const int m = w == W - 1 ? 0 : w + 1;
        double u = 0.0, p = 1.0;
        for (int k = 0, j = m; k < W; ++k) {
            u += p * ends[j][lane];
            p *= j == W - 1 ? zLast : zS;
            j = j == W - 1 ? 0 : j + 1;
        }
        u /= 1.0 - zN;
        double q = z;
#pragma unroll
        for (int i = S - 1; i >= 0; --i) {
            if (i < L) { r[i] = scale * (r[i] + q * u); q *= z; }
        }
    }
    // the sink, in runs of SR points (shorter runs where more waves share the
    // registers)
    constexpr int SR = MAXW > 8 ? 8 : 16;
#pragma unroll
    for (int h = 0; h < S; h += SR) {
        unsigned o[SR];
        double v[SR];
        bool ok[SR];
#pragma unroll
        for (int m = 0; m < SR; ++m) {
            o[m] = base + (unsigned)(s0 + h + m) * sa;
            v[m] = r[h + m];
            ok[m] = active && h + m < L;
        }
        sink_run<SR>(sink, o, v, ok);
    }
}

// Compact derivative along x of rows of at most 12 * kSegLen = 384 points, the
// row-wise counterpart of k_compact_seg.  Each wavefront stages RW rows in
// LDS with coalesced loads; lane l then solves segment s = l % NS (NS = the
// segments per row) of row l / NS from LDS, the periodic carries between the
// segments of a row coming from the other lanes of that row by cross-lane
// reads.  The results go back to LDS and leave through coalesced stores
// (element offsets in 32 bits: launched for N < 2^29).
// Row layout in LDS: point x at x + x / 32 (a one-element skew per segment)
// in rows of P doubles, P = 8 (mod 16), so the lanes of a half-wave read
// different banks.
struct XSegGeom {
    int n, NS, RW, P;     // row length, segments per row, rows per wave, LDS row stride
    unsigned magic;       // e / n == (e * magic) >> 20 for 0 <= e < 2048 (n < 512)
};

inline XSegGeom xseg_geom(int n)
{
    XSegGeom q;
    q.n = n;
    q.NS = (n + kSegLen - 1) / kSegLen;
    q.RW = 64 / q.NS;
    q.P = (n + q.NS + 7) / 16 * 16 + 8;
    q.magic = ((1u << 20) + (unsigned)n - 1) / (unsigned)n;
    return q;
}

__global__ void __launch_bounds__(256) k_compact_xseg(const double* __restrict__ f, CompactSink sink,
                                                      long long nrows, XSegGeom q, Compact c, double z,
                                                      double scale, double zS, double zLast, double zN)
{
    extern __shared__ double xrows[];
    constexpr int S = kSegLen;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int n = q.n, NS = q.NS, RW = q.RW, P = q.P;
    double* rows = xrows + (size_t)wv * RW * P;
    const long long row0 = ((long long)blockIdx.x * (blockDim.x >> 6) + wv) * RW;
    // the wave's RW * n <= 2048 points: element e = lane + 64 m of the rows
    // laid end to end; all loads first, then the LDS writes
    {
        double t[32];
#pragma unroll
        for (int m = 0; m < 32; ++m) {
            const unsigned e = (unsigned)(lane + 64 * m);
            const unsigned j = (e * q.magic) >> 20, x = e - j * (unsigned)n;
            t[m] = (int)j < RW && row0 + j < nrows ? f[(unsigned)((row0 + j) * n) + x] : 0.0;
        }
#pragma unroll
        for (int m = 0; m < 32; ++m) {
            const unsigned e = (unsigned)(lane + 64 * m);
            const unsigned j = (e * q.magic) >> 20, x = e - j * (unsigned)n;
            if ((int)j < RW) rows[j * P + x + x / S] = t[m];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // this lane's segment; lanes past RW * NS work on a copy of row 0 and
    // store nothing
    const int jr = lane / NS < RW ? lane / NS : 0;
    const int sg = lane % NS;
    const bool mine = lane / NS < RW && row0 + jr < nrows;
    const int s0 = sg * S;
    const int L = min(S, n - s0);
    const double* rr = rows + jr * P;
    const double ha = 0.5 * c.ca, hb = 0.25 * c.cb, hc = c.cc / 6.0;
    double r[S + 6];
#pragma unroll
    for (int k = 0; k < S + 6; ++k) {
        int x = s0 - 3 + k;             // in [-3, n + 2]; n >= 4
        x += x < 0 ? n : 0;
        x -= x >= n ? n : 0;
        r[k] = k < L + 6 ? rr[x + x / S] : 0.0;
    }
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        if (i < L) {
            const double v = ha * (r[i + 4] - r[i + 2]) + hb * (r[i + 5] - r[i + 1]) + hc * (r[i + 6] - r[i]);
            acc = v + z * acc;
            r[i] = acc;
        }
    }
    const int rl = (lane / NS) * NS;    // first lane of this row's segments
    {
        double t = 0.0, p = 1.0;
        const int m = sg == 0 ? NS - 1 : sg - 1;
        for (int k = 0, j = m; k < NS; ++k) {
            t += p * __shfl(acc, rl + j, 64);
            p *= j == NS - 1 ? zLast : zS;
            j = j == 0 ? NS - 1 : j - 1;
        }
        t /= 1.0 - zN;
        double qz = z;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (i < L) { r[i] += qz * t; qz *= z; }
        }
    }
    acc = 0.0;
#pragma unroll
    for (int i = S - 1; i >= 0; --i) {
        if (i < L) { acc = r[i] + z * acc; r[i] = acc; }
    }
    {
        double u = 0.0, p = 1.0;
        const int m = sg == NS - 1 ? 0 : sg + 1;
        for (int k = 0, j = m; k < NS; ++k) {
            u += p * __shfl(acc, rl + j, 64);
            p *= j == NS - 1 ? zLast : zS;
            j = j == NS - 1 ? 0 : j + 1;
        }
        u /= 1.0 - zN;
        double qz = z;
        // every lane has read its inputs (program order within the wavefront)
        double* wr = rows + jr * P;
#pragma unroll
        for (int i = S - 1; i >= 0; --i) {
            if (i < L) {
                if (mine) wr[s0 + i + (s0 + i) / S] = scale * (r[i] + qz * u);
                qz *= z;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int h = 0; h < 32; h += 16) {
        unsigned o[16];
        double v[16];
        bool ok[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const unsigned e = (unsigned)(lane + 64 * (h + m));
            const unsigned j = (e * q.magic) >> 20, x = e - j * (unsigned)n;
            ok[m] = (int)j < RW && row0 + j < nrows;
            o[m] = ok[m] ? (unsigned)((row0 + j) * n) + x : 0u;
            v[m] = ok[m] ? rows[j * P + x + x / S] : 0.0;
        }
        sink_run<16>(sink, o, v, ok);
    }
}

// Compact derivative along x (unit stride) of whole rows: one wavefront per
// row, lanes along x.  The row is first staged in LDS (all its loads in
// flight at once).  Both recursions then run as wavefront-wide scans over
// chunks of 64 consecutive points (a_i = v_i + z a_{i-1} in log2(64) shuffle
// steps, plus z^(lane+1) times the carry from the previous chunk).  The sweep
// starts W >= K points early (periodic positions); the forward results of the
// row replace nothing and sit in a second LDS row for the backward sweep.
constexpr int kScanWarm = 128;

__global__ void __launch_bounds__(256) k_compact_x(const double* __restrict__ f, CompactSink sink, int nx,
                                                   long long nrows, Compact c, double z, double scale)
{
    extern __shared__ double wrow[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const long long row = (long long)blockIdx.x * (blockDim.x >> 6) + wv;
    if (row >= nrows) return;   // whole wavefront leaves; no block barrier below
    double* fr = wrow + (size_t)wv * 2 * nx;   // the row of f
    double* wb = fr + nx;                       // forward results
    for (int x = lane; x < nx; x += 64) fr[x] = f[row * nx + x];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double ha = 0.5 * c.ca, hb = 0.25 * c.cb, hc = c.cc / 6.0;
    double zs[7];    // z^(2^s)
    zs[0] = z;
#pragma unroll
    for (int s = 1; s < 7; ++s) zs[s] = zs[s - 1] * zs[s - 1];
    double zl = 1.0;  // z^(lane+1) from the binary digits of lane+1
#pragma unroll
    for (int s = 0; s < 7; ++s)
        if ((lane + 1) >> s & 1) zl *= zs[s];
    auto scan = [&](double a, double carry) {
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const double t = __shfl_up(a, 1u << s, 64);
            if (lane >= (1 << s)) a += zs[s] * t;
        }
        return a + zl * carry;
    };
    // forward sweep over positions -W .. nx-1
    double carry = 0.0;
    for (int p0 = -kScanWarm; p0 < nx; p0 += 64) {
        const int p = p0 + lane;
        const bool valid = p < nx;
        double v = 0.0;
        int x = 0;
        if (valid) {
            x = pmod(p, nx);
            const int x1 = wrapc(x + 1, nx), x_1 = wrapc(x - 1, nx);
            const int x2 = pmod(x + 2, nx), x_2 = pmod(x - 2, nx);
            const int x3 = pmod(x + 3, nx), x_3 = pmod(x - 3, nx);
            v = ha * (fr[x1] - fr[x_1]) + hb * (fr[x2] - fr[x_2]) + hc * (fr[x3] - fr[x_3]);
        }
        const double a = scan(v, carry);
        carry = __shfl(a, 63, 64);
        if (valid && p >= 0) wb[x] = a;
    }
    // backward sweep over positions nx-1+W .. 0 (lane order = descending);
    // the results replace the row of f in LDS
    carry = 0.0;
    for (int q0 = nx - 1 + kScanWarm; q0 >= 0; q0 -= 64) {
        const int q = q0 - lane;
        const bool valid = q >= 0;
        const int x = valid ? pmod(q, nx) : 0;
        const double a = scan(valid ? wb[x] : 0.0, carry);
        carry = __shfl(a, 63, 64);
        if (valid && q < nx) fr[x] = scale * a;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the sink in runs of 16 points per lane, loads before stores
    for (int x0 = 0; x0 < nx; x0 += 64 * 16) {
        long long o[16];
        double v[16];
        bool ok[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int x = x0 + lane + 64 * m;
            ok[m] = x < nx;
            o[m] = row * nx + (ok[m] ? x : 0);
            v[m] = ok[m] ? fr[x] : 0.0;
        }
        sink_run<16, long long>(sink, o, v, ok);
    }
}

// ---------------------------------------------------------------------------
// Memory ceiling of the step's access pattern (a measurement, not a step):
// Q population arrays of N doubles copied node by node, either aligned
// (dst_i(x) = src_i(x)) or as the lattice's pull (dst_i(x) = src_i(x - e_i),
// periodic), with no arithmetic.  The rate it reaches bounds any SoA step
// that reads and writes every population once.
// ---------------------------------------------------------------------------
template <int LAT, bool PULL>
__global__ void __launch_bounds__(256) k_probe_copy(const double* __restrict__ src, double* __restrict__ dst, Grid g)
{
    using L = Lat<LAT>;
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    coords(n, g, x, y, z);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        long long s = n;
        if constexpr (PULL) {
            const int xs = wrapc(x - L::ex(i), g.nx), ys = wrapc(y - L::ey(i), g.ny);
            const int zs = LAT == 1 ? wrapc(z - L::ez(i), g.nz) : 0;
            s = (long long)zs * g.nxy + (long long)ys * g.nx + xs;
        }
        dst[(long long)i * g.ps + n] = src[(long long)i * g.ps + s];
    }
}

}  // namespace lbm
