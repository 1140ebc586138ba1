// lbm_fused.hpp -- fused collide kernels that also produce the next density.
//
// The step needs rho(t) at every node within the stencil halo before any
// collision, and rho(t+1)(x) = sum_i f*_i(x - e_i) depends on the collisions of
// x's neighbours.  Instead of a separate pass that re-reads all Q populations
// to form rho(t+1), each workgroup collides its tile plus a one-node ring in x
// and y (the ring nodes are collided but not stored), exchanges the
// post-collision populations through LDS, and writes rho(t+1) for its tile.
// In 3D the workgroup marches along z through a segment of planes; the z
// neighbours' contributions arrive from the previous and next plane of the
// march, one extra plane at each end of the segment.
//
// Per node the kernel reads the Q populations once (plus the ring, mostly
// cache hits), rho and mu_hat (stencil halos from cache) and writes Q
// populations and rho(t+1).  mu_hat comes from the small k_mu pass.
#pragma once

#include <hip/hip_runtime.h>
#include "lbm_kernels.hpp"

namespace lbm {

constexpr int FX = 64;   // tile width (x)
constexpr int FY3 = 4;   // tile height (y), 3D
constexpr int FY2 = 4;   // tile height (y), 2D
constexpr int FZ = 32;   // z planes per segment, 3D
constexpr int FTH3 = (FX + 2) * (FY3 + 2);   // 396 threads
constexpr int FTH2 = (FX + 2) * (FY2 + 2);   // 396 threads

struct TileGeom {
    int ntx, nty, nsz;   // tiles along x, y and z segments
};

// LDS slot of direction i for the post-collision exchange (-1: direction with
// no in-plane shift, kept in registers).  D2Q9: the eight moving directions;
// D3Q19: all but the rest and the two pure z links (i = 5, 6).
template <int LAT>
__host__ __device__ constexpr int xcls_of(int i)
{
    return LAT == 0 ? i - 1 : (i == 0 || i == 5 || i == 6) ? -1 : (i <= 4 ? i - 1 : i - 3);
}

__device__ __forceinline__ int pwrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Fused collide for the per-axis explicit schemes (CD2/CD4/CD6).  Thread
// (lx, ly) owns column (x0-1+lx, y0-1+ly) of the tile plus its ring.  Per
// plane of the march the workgroup stages rho and mu_hat of the plane (tile,
// ring and an R-wide halo) in LDS for the in-plane stencil arms; the z arms
// come from per-thread register queues of the thread's own column.
template <int LAT, int SCH, int TY, int OCC, bool PIPE>
__global__ void __launch_bounds__((FX + 2) * (TY + 2), OCC)
k_fused(const double* __restrict__ S, double* __restrict__ Sn, const double* __restrict__ rho,
        const double* __restrict__ mu, double* __restrict__ rho_next, Grid g, TileGeom tg, double one_m_omega)
{
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    constexpr int R = radius(SCH);
    constexpr int W = FX + 2, H = TY + 2, NTH = W * H;
    constexpr int WR = W + 2 * R, HR = H + 2 * R;
    constexpr int NCL = LAT == 1 ? 16 : 8;
    constexpr int QZ = LAT == 1 ? 2 * R + 1 : 1;
    constexpr double cs2 = 1.0 / 3.0;
    __shared__ double xs[NCL][NTH];
    __shared__ double rp[HR * WR];
    __shared__ double mp[HR * WR];

    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int nxy = (int)g.nxy, N = (int)g.N;
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous run of tiles so neighbouring tiles (ring and halo reads)
    // share an L2.
    int b = blockIdx.x;
    {
        const int nb = gridDim.x, per = nb / 8;
        if (b < per * 8) b = (b % 8) * per + b / 8;
    }
    const int tx = b % tg.ntx;
    const int ty = (b / tg.ntx) % tg.nty;
    const int sz = b / (tg.ntx * tg.nty);
    const int x0 = tx * FX, y0 = ty * TY;
    const int wx = min(FX, nx - x0), wy = min(TY, ny - y0);
    const int lid = threadIdx.x;
    const int lx = lid % W, ly = lid / W;
    const bool active = lx <= wx + 1 && ly <= wy + 1;
    const bool inner = lx >= 1 && lx <= wx && ly >= 1 && ly <= wy;
    const int x = active ? wrapc(x0 - 1 + lx, nx) : 0;
    const int y = active ? wrapc(y0 - 1 + ly, ny) : 0;
    const int xm = wrapc(x - 1, nx), xp = wrapc(x + 1, nx);
    const int yc = y * nx, ym = wrapc(y - 1, ny) * nx, yp = wrapc(y + 1, ny) * nx;
    const int z0 = LAT == 1 ? sz * FZ : 0;
    const int z1 = LAT == 1 ? min(z0 + FZ, nz) : 1;
    const int c0 = (ly + R) * WR + (lx + R);   // own position in the staged plane

    // z queues of rho and mu_hat for the own column: index k <-> plane z-R+k
    double qr[QZ], qm[QZ];
#pragma unroll
    for (int k = 0; k < QZ; ++k) { qr[k] = 0.0; qm[k] = 0.0; }
    if constexpr (LAT == 1) {
        if (active) {
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) {
                const int zz = pwrap(z0 - 1 - R + k, nz);
                qr[k + 1] = rho[zz * nxy + yc + x];
                qm[k + 1] = mu[zz * nxy + yc + x];
            }
        }
    }

    // pull f_i(x) = S_i(x - e_i) of the own column at plane z
    auto pull_plane = [&](int z, double (&f)[Q]) {
        const int zo = z * nxy;
        const int zmo = LAT == 1 ? wrapc(z - 1, nz) * nxy : 0;
        const int zpo = LAT == 1 ? wrapc(z + 1, nz) * nxy : 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int ox = L::ex(i) == 1 ? xm : L::ex(i) == -1 ? xp : x;
            const int oy = L::ey(i) == 1 ? ym : L::ey(i) == -1 ? yp : yc;
            const int oz = L::ez(i) == 1 ? zmo : L::ez(i) == -1 ? zpo : zo;
            f[i] = S[(long long)i * N + (oz + oy + ox)];
        }
    };

    double acc_m1 = 0.0, acc_0 = 0.0;
    const int zb = LAT == 1 ? z0 - 1 : 0, ze = LAT == 1 ? z1 : 0;
    double fnext[PIPE ? Q : 1];
    if constexpr (PIPE) {
        if (active) pull_plane(LAT == 1 ? pwrap(zb, nz) : 0, fnext);
    }
    for (int zr = zb; zr <= ze; ++zr) {
        const int z = LAT == 1 ? pwrap(zr, nz) : 0;
        const int zo = z * nxy;
        // pulls of this plane: issued before the staging (no dependence), or,
        // pipelined, already in flight since the previous plane's compute
        double f[Q];
        if constexpr (PIPE) {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = fnext[i];
        } else if (active) {
            pull_plane(z, f);
        }
        // stage the plane (tile + ring + R halo) of rho and mu_hat
        for (int idx = lid; idx < HR * WR; idx += NTH) {
            const int hy = idx / WR, hx = idx - hy * WR;
            const int o = zo + pwrap(y0 - 1 - R + hy, ny) * nx + pwrap(x0 - 1 - R + hx, nx);
            rp[idx] = rho[o];
            mp[idx] = mu[o];
        }
        if constexpr (LAT == 1) {
#pragma unroll
            for (int k = 0; k < QZ - 1; ++k) { qr[k] = qr[k + 1]; qm[k] = qm[k + 1]; }
            if (active) {
                const int zz = pwrap(zr + R, nz) * nxy + yc + x;
                qr[QZ - 1] = rho[zz];
                qm[QZ - 1] = mu[zz];
            }
        }
        __syncthreads();
        if constexpr (PIPE) {
            // next plane's pulls go out now and land during this plane's compute
            if (active && zr < ze) pull_plane(LAT == 1 ? pwrap(zr + 1, nz) : 0, fnext);
        }
        double own_m1 = 0.0, own_0 = 0.0, own_p1 = 0.0;   // post-collision values without in-plane shift
        if (active) {
            double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                r += f[i];
                jx += L::ex(i) * f[i]; jy += L::ey(i) * f[i]; jz += L::ez(i) * f[i];
            }
            double grx = 0.0, gry = 0.0, grz = 0.0, gmx = 0.0, gmy = 0.0, gmz = 0.0;
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                const double c = d1(SCH, m);
                grx += c * (rp[c0 + m] - rp[c0 - m]);
                gry += c * (rp[c0 + m * WR] - rp[c0 - m * WR]);
                gmx += c * (mp[c0 + m] - mp[c0 - m]);
                gmy += c * (mp[c0 + m * WR] - mp[c0 - m * WR]);
                if constexpr (LAT == 1) {
                    grz += c * (qr[R + m] - qr[R - m]);
                    gmz += c * (qm[R + m] - qm[R - m]);
                }
            }
            const double Fx = -r * gmx + cs2 * grx, Fy = -r * gmy + cs2 * gry, Fz = -r * gmz + cs2 * grz;
            // collision (Eq 1 SRT, Eq 6, Eq 8), each post-collision value stored
            // as soon as it is formed
            const double ir = 1.0 / r;
            const double ux = jx * ir, uy = jy * ir, uz = jz * ir;
            const double vx = ux + Fx * ir, vy = uy + Fy * ir, vz = uz + Fz * ir;
            const double uu = 1.0 - 1.5 * (ux * ux + uy * uy + uz * uz);
            const double vv = 1.0 - 1.5 * (vx * vx + vy * vy + vz * vz);
            const bool store = inner && zr >= z0 && zr < z1;
            const int n = zo + yc + x;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double wr = L::w(i) * r;
                const double eu = L::ex(i) * ux + L::ey(i) * uy + L::ez(i) * uz;
                const double ev = L::ex(i) * vx + L::ey(i) * vy + L::ez(i) * vz;
                const double fe = wr * (uu + eu * (3.0 + 4.5 * eu));
                const double fv = wr * (vv + ev * (3.0 + 4.5 * ev));
                const double o = fv + one_m_omega * (f[i] - fe);
                if (store) Sn[(long long)i * N + n] = o;
                if (xcls_of<LAT>(i) >= 0) xs[xcls_of<LAT>(i)][lid] = o;
                else if (L::ez(i) == -1) own_m1 = o;
                else if (L::ez(i) == 0) own_0 = o;
                else own_p1 = o;
            }
        }
        __syncthreads();
        if (inner) {
            double a_m1 = own_m1, a_0 = own_0, a_p1 = own_p1;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (xcls_of<LAT>(i) < 0) continue;
                const double v = xs[xcls_of<LAT>(i)][(ly - L::ey(i)) * W + (lx - L::ex(i))];
                if (L::ez(i) == -1) a_m1 += v; else if (L::ez(i) == 0) a_0 += v; else a_p1 += v;
            }
            if constexpr (LAT == 1) {
                acc_m1 += a_m1;
                if (zr - 1 >= z0 && zr - 1 < z1) rho_next[(zr - 1) * nxy + yc + x] = acc_m1;
                acc_m1 = acc_0 + a_0;
                acc_0 = a_p1;
            } else {
                rho_next[yc + x] = a_0;
            }
        }
    }
}

// The fused path covers the per-axis explicit schemes on grids whose node
// count fits 32-bit offsets.
template <int LAT, int SCH>
inline bool fused_available(const Grid& g) { return (SCH == CD2 || SCH == CD4 || SCH == CD6) && g.N < (1LL << 31); }

// Launch variants of the fused kernel (tile height, waves per SIMD the register
// allocation must allow).  The tuner times them on the actual grid.
struct FusedVariant { int ty, occ, pipe; };
constexpr FusedVariant kFusedVariants[] = { {8, 2, 0}, {4, 3, 0}, {6, 3, 0}, {4, 2, 1}, {5, 2, 1}, {3, 2, 1} };
constexpr int kNumFusedVariants = 6;

inline TileGeom fused_tiles(int ty, const Grid& g, bool three_d)
{
    TileGeom t;
    t.ntx = (g.nx + FX - 1) / FX;
    t.nty = (g.ny + ty - 1) / ty;
    t.nsz = three_d ? (g.nz + FZ - 1) / FZ : 1;
    return t;
}

template <int LAT, int SCH, int TY, int OCC, bool PIPE>
inline void launch_fused_v(const double* S, double* Sn, const double* rho, const double* mu, double* rho_next,
                           const Grid& g, double one_m_omega, hipStream_t st)
{
    const TileGeom t = fused_tiles(TY, g, LAT == 1);
    const unsigned nb = (unsigned)(t.ntx * t.nty * t.nsz);
    hipLaunchKernelGGL((k_fused<LAT, SCH, TY, OCC, PIPE>), dim3(nb), dim3((FX + 2) * (TY + 2)), 0, st, S, Sn, rho, mu,
                       rho_next, g, t, one_m_omega);
}

template <int LAT, int SCH>
inline void launch_fused_collide(int variant, const double* S, double* Sn, const double* rho, const double* mu,
                                 double* rho_next, const Grid& g, double one_m_omega, hipStream_t st)
{
    switch (variant) {
    case 1: launch_fused_v<LAT, SCH, 4, 3, false>(S, Sn, rho, mu, rho_next, g, one_m_omega, st); break;
    case 2: launch_fused_v<LAT, SCH, 6, 3, false>(S, Sn, rho, mu, rho_next, g, one_m_omega, st); break;
    case 3: launch_fused_v<LAT, SCH, 4, 2, true>(S, Sn, rho, mu, rho_next, g, one_m_omega, st); break;
    case 4: launch_fused_v<LAT, SCH, 5, 2, true>(S, Sn, rho, mu, rho_next, g, one_m_omega, st); break;
    case 5: launch_fused_v<LAT, SCH, 3, 2, true>(S, Sn, rho, mu, rho_next, g, one_m_omega, st); break;
    default: launch_fused_v<LAT, SCH, 8, 2, false>(S, Sn, rho, mu, rho_next, g, one_m_omega, st); break;
    }
}

}  // namespace lbm
