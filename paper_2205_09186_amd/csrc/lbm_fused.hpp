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
    int mz;              // planes per z segment (marching stencil kernels)
};

inline TileGeom fused_tiles(int ty, const Grid& g, bool three_d)
{
    TileGeom t;
    t.ntx = (g.nx + FX - 1) / FX;
    t.nty = (g.ny + ty - 1) / ty;
    t.nsz = three_d ? (g.nz + FZ - 1) / FZ : 1;
    t.mz = FZ;
    return t;
}

// LDS slot of direction i for the post-collision exchange (-1: direction with
// no in-plane shift, kept in registers).  D2Q9: the eight moving directions;
// D3Q19: all but the rest and the two pure z links (i = 5, 6).
template <int LAT>
__host__ __device__ constexpr int xcls_of(int i)
{
    return LAT == 0 ? i - 1 : (i == 0 || i == 5 || i == 6) ? -1 : (i <= 4 ? i - 1 : i - 3);
}

// Load / store at a 32-bit element index from a base pointer the whole
// workgroup shares: the zero-extended byte offset lets the compiler use the
// scalar-base + 32-bit vector-offset addressing form (one VGPR per access
// instead of a 64-bit address).  Requires fewer than 2^29 nodes per buffer.
__device__ __forceinline__ double ld32(const double* base, unsigned idx)
{
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + (size_t)(idx * 8u));
}
__device__ __forceinline__ void st32(double* base, unsigned idx, double v)
{
    *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + (size_t)(idx * 8u)) = v;
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
// FULL: SRT with tau = 1 (one_m_omega == 0), where f* = feq(rho, u + du) exactly and
// the pulled populations are dead once the moments are formed.
template <int LAT, int SCH, int TY, int OCC, bool PIPE, bool FULL>
__global__ void __launch_bounds__((FX + 2) * (TY + 2), OCC)
k_fused(const double* __restrict__ S, double* __restrict__ Sn, const double* __restrict__ rho,
        const double* __restrict__ mu, double* __restrict__ rho_next, Grid g, TileGeom tg, Relax rx)
{
    const double one_m_omega = rx.omo;
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
            f[i] = ld32(S + (long long)i * g.ps, (unsigned)(oz + oy + ox));
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
            const unsigned o = (unsigned)(zo + pwrap(y0 - 1 - R + hy, ny) * nx + pwrap(x0 - 1 - R + hx, nx));
            rp[idx] = ld32(rho, o);
            mp[idx] = ld32(mu, o);
        }
        if constexpr (LAT == 1) {
#pragma unroll
            for (int k = 0; k < QZ - 1; ++k) { qr[k] = qr[k + 1]; qm[k] = qm[k + 1]; }
            if (active) {
                const unsigned zz = (unsigned)(pwrap(zr + R, nz) * nxy + yc + x);
                qr[QZ - 1] = ld32(rho, zz);
                qm[QZ - 1] = ld32(mu, zz);
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
            double om[LAT == 0 ? 9 : 1];   // MRT post-collision values (D2Q9)
            if constexpr (LAT == 0 && !FULL) {
                if (rx.mrt) {
                    double fe[9], fv[9];
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        const double wr = L::w(i) * r;
                        const double eu = L::ex(i) * ux + L::ey(i) * uy;
                        const double ev = L::ex(i) * vx + L::ey(i) * vy;
                        fe[i] = wr * (uu + eu * (3.0 + 4.5 * eu));
                        fv[i] = wr * (vv + ev * (3.0 + 4.5 * ev));
                    }
                    mrt_post(f, fe, fv, rx, om);
                }
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double wr = L::w(i) * r;
                const double eu = L::ex(i) * ux + L::ey(i) * uy + L::ez(i) * uz;
                const double ev = L::ex(i) * vx + L::ey(i) * vy + L::ez(i) * vz;
                const double fe = wr * (uu + eu * (3.0 + 4.5 * eu));
                const double fv = wr * (vv + ev * (3.0 + 4.5 * ev));
                double o = FULL ? fv : fv + one_m_omega * (f[i] - fe);
                if constexpr (LAT == 0 && !FULL) {
                    if (rx.mrt) o = om[i];
                }
                (void)fe;
                if (store) st32(Sn + (long long)i * g.ps, (unsigned)n, o);
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
                if (zr - 1 >= z0 && zr - 1 < z1) st32(rho_next, (unsigned)((zr - 1) * nxy + yc + x), acc_m1);
                acc_m1 = acc_0 + a_0;
                acc_0 = a_p1;
            } else {
                rho_next[yc + x] = a_0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Stencil marches over 64 x 8 tiles for the per-axis explicit schemes.  Per
// plane, the tile plus its R-wide in-plane halo of each input field is staged
// in LDS (double-buffered: one barrier per plane); the z arms come from a
// per-thread register queue of the own column.  The global loads of the next
// plane are issued before the current plane is computed, so their latency
// overlaps the barrier and the arithmetic.  Per node: one HBM read of each
// input and one write of each output; the halo re-reads hit L2.
//   NF = 1: mu_hat = k^2 psi'(rho) - kappa_hat lap(rho) (Eq 15, Eq 16), with
//           the summation order of lap_at.
//   NF = 2: F = -rho grad(mu_hat) + cs^2 grad(rho) (Eq 12), gradients summed
//           as in grad_at; F stored as three (two in 2D) planes of N.
// ---------------------------------------------------------------------------
// Tiles of MX x MY (the force march of the CD schemes in 3D: MX x 16, which
// doubles the waves per CU that its LDS ring of planes allows; 0.157 -> 0.138
// ms on 256^3 CD6).
constexpr int MX = 64, MY = 8, MZ = 32;

inline TileGeom march_tiles(const Grid& g, bool three_d, int mz, int my = MY)
{
    TileGeom t;
    t.ntx = (g.nx + MX - 1) / MX;
    t.nty = (g.ny + my - 1) / my;
    t.mz = mz;
    t.nsz = three_d ? (g.nz + mz - 1) / mz : 1;
    return t;
}

template <int DIM, int SCH, int NF, int TYM = MY>
__global__ void __launch_bounds__(MX * TYM) k_march(const double* __restrict__ rho, const double* __restrict__ mu,
                                                    double* __restrict__ out, Grid g, TileGeom tg, Eos e)
{
    constexpr int R = radius(SCH);
    constexpr int WR = MX + 2 * R, HR = TYM + 2 * R, CELLS = WR * HR, NTH = MX * TYM;
    constexpr int SPT = (CELLS + NTH - 1) / NTH;
    // Two ways to feed the z arms.  NF = 1 (mu_hat, arithmetic-bound): the
    // own column's plane p + R comes from global memory with the prefetch and
    // plane p is computed from a double-buffered stage.  NF = 2 (force, two
    // fields): every plane is loaded once, staged when it enters the march,
    // and the own column is pushed from LDS; plane p - R is computed from its
    // slot, and R + 2 slots keep each read ahead of the overwrite that follows
    // the next barrier.
    // The isotropic schemes (Eq 25) reach diagonal neighbours in z as well:
    // all 2R + 1 planes of the stencil are staged (2R + 2 slots), the march
    // starts R planes early and every arm is read from LDS.
    constexpr bool ISO = is_iso(SCH);
    constexpr bool SLOTS = DIM == 3 && (NF == 2 || ISO);
    constexpr int LAG = SLOTS ? R : 0;
    constexpr int NS = SLOTS ? (ISO ? 2 * R + 2 : R + 2) : 2;
    constexpr int QZ = DIM == 3 ? 2 * R + 1 : 1;
    constexpr double cs2 = 1.0 / 3.0;
    __shared__ double sp[NS][NF][CELLS];

    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int nxy = (int)g.nxy;
    const unsigned N = (unsigned)g.N;
    int b = blockIdx.x;
    {
        const int nb = gridDim.x, per = nb / 8;
        if (b < per * 8) b = (b % 8) * per + b / 8;
    }
    const int tx = b % tg.ntx;
    const int ty = (b / tg.ntx) % tg.nty;
    const int sz = b / (tg.ntx * tg.nty);
    const int x0 = tx * MX, y0 = ty * TYM;
    const int lid = threadIdx.x;
    const int lx = lid % MX, ly = lid / MX;
    const bool in = lx < min(MX, nx - x0) && ly < min(TYM, ny - y0);
    const int col = in ? (y0 + ly) * nx + x0 + lx : 0;
    const int z0 = DIM == 3 ? sz * tg.mz : 0;
    const int z1 = DIM == 3 ? min(z0 + tg.mz, nz) : 1;
    const int c0 = (ly + R) * WR + (lx + R);
    const double* src[2] = { rho, mu };

    // in-plane offsets of the staged cells this thread loads (fixed over the march)
    unsigned off[SPT];
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int idx = lid + k * NTH;
        const int hy = idx / WR, hx = idx - hy * WR;
        off[k] = idx < CELLS ? (unsigned)(pwrap(y0 - R + hy, ny) * nx + pwrap(x0 - R + hx, nx)) : 0u;
    }
    // z queue of the own column, index k <-> plane z - R + k for the plane z
    // computed next.  Planes before the first staged one are loaded here.
    double q[NF][QZ];
    // 3D isotropic schemes: sums pending for the output planes p - R .. p + R
    // (index j <-> plane p - R + j), fed by each staged plane once
    constexpr bool PUSH = ISO && DIM == 3;
    constexpr int NA = NF == 1 ? 1 : 6;
    double A[PUSH ? 2 * R + 1 : 1][NA];
#pragma unroll
    for (int j = 0; j < (PUSH ? 2 * R + 1 : 1); ++j)
#pragma unroll
        for (int a = 0; a < NA; ++a) A[j][a] = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int k = 0; k < QZ; ++k) q[f][k] = 0.0;
    if constexpr (DIM == 3 && !ISO) {
        if (in) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int k = SLOTS ? R : 0; k < 2 * R; ++k)
                    q[f][k + 1] = ld32(src[f], (unsigned)(pwrap(z0 - R - LAG + k, nz) * nxy + col));
        }
    }
    double sv[NF][SPT], qn[NF];
    auto fetch = [&](int p) {
        const unsigned zo = (unsigned)(pwrap(p, nz) * nxy);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int k = 0; k < SPT; ++k)
                if (lid + k * NTH < CELLS) sv[f][k] = ld32(src[f], zo + off[k]);
            if constexpr (DIM == 3 && !SLOTS) {
                if (in) qn[f] = ld32(src[f], (unsigned)(pwrap(p + R, nz) * nxy + col));
            }
        }
    };
    const int pe = z1 - 1 + LAG;                        // last plane staged
    const int pb = DIM == 3 && ISO ? z0 - R : z0;       // first plane staged
    fetch(pb);
    for (int p = pb; p <= pe; ++p) {
        double (*s)[CELLS] = sp[(p - pb) % NS];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int k = 0; k < SPT; ++k)
                if (lid + k * NTH < CELLS) s[f][lid + k * NTH] = sv[f][k];
        if constexpr (DIM == 3 && !SLOTS) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
#pragma unroll
                for (int k = 0; k < QZ - 1; ++k) q[f][k] = q[f][k + 1];
                q[f][QZ - 1] = qn[f];
            }
        }
        if (p < pe) fetch(p + 1);
        // NF = 1, CD schemes in 3D: the own node's bulk potential comes from
        // its z queue, so it is evaluated before the barrier, while the next
        // plane's loads are in flight (0.117 -> 0.111 ms on 256^3 CD6)
        double mb = 0.0;
        if constexpr (NF == 1 && DIM == 3 && !ISO) {
            if (in) mb = mu_bulk(q[0][R], e);
        }
        __syncthreads();
        if constexpr (SLOTS && !ISO) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
#pragma unroll
                for (int k = 0; k < QZ - 1; ++k) q[f][k] = q[f][k + 1];
                q[f][QZ - 1] = s[f][c0];
            }
        }
        if constexpr (PUSH) {
            // each in-plane neighbour of plane p is read once and added, with
            // the weight of Eq 25 for every z offset it has, to the outputs
            // it reaches; the output plane p - R is then complete
            if (in) {
                const int sl = (p - pb) % NS;
#pragma unroll
                for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) {
                        double v[NF];
#pragma unroll
                        for (int f = 0; f < NF; ++f) v[f] = sp[sl][f][c0 + dy * WR + dx];
#pragma unroll
                        for (int dz = -R; dz <= R; ++dz) {
                            const int sh = dx * dx + dy * dy + dz * dz;
                            const double w = iso_w(DIM, SCH, sh);
                            if (sh == 0 || w == 0.0) continue;
                            // the neighbour at +dz of output plane p - dz
                            double* a = A[R - dz];
                            if constexpr (NF == 1) {
                                a[0] += w * v[0];
                            } else {
                                if (dx) { a[0] += (dx * w) * v[0]; a[3] += (dx * w) * v[1]; }
                                if (dy) { a[1] += (dy * w) * v[0]; a[4] += (dy * w) * v[1]; }
                                if (dz) { a[2] += (dz * w) * v[0]; a[5] += (dz * w) * v[1]; }
                            }
                        }
                    }
                const int z = p - R;
                if (z >= z0) {
                    const unsigned n = (unsigned)(z * nxy + col);
                    const double c = sp[(z - pb) % NS][0][c0];   // rho at the output node
                    if constexpr (NF == 1) {
                        double wsum = 0.0;   // sum of the weights over the stencil
#pragma unroll
                        for (int dz = -R; dz <= R; ++dz)
#pragma unroll
                            for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                                for (int dx = -R; dx <= R; ++dx) {
                                    const int sh = dx * dx + dy * dy + dz * dz;
                                    if (sh) wsum += iso_w(DIM, SCH, sh);
                                }
                        st32(out, n, mu_bulk(c, e) - e.kappa * (2.0 * (A[0][0] - wsum * c)));
                    } else {
                        st32(out, n, -c * A[0][3] + cs2 * A[0][0]);
                        st32(out + N, n, -c * A[0][4] + cs2 * A[0][1]);
                        st32(out + 2 * (size_t)N, n, -c * A[0][5] + cs2 * A[0][2]);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 2 * R; ++j)
#pragma unroll
                for (int a = 0; a < NA; ++a) A[j][a] = A[j + 1][a];
#pragma unroll
            for (int a = 0; a < NA; ++a) A[2 * R][a] = 0.0;
            continue;
        }
        if (p < z0 + LAG || !in) continue;
        const int z = p - LAG;
        double (*c)[CELLS] = sp[(z - pb) % NS];
        const unsigned n = (unsigned)(z * nxy + col);
        if constexpr (ISO) {
            // the stencil of lap_at / grad_at (Eq 25), shell weights by |e|^2,
            // planes z - R .. z + R from their slots
            constexpr int RZ = DIM == 3 ? R : 0;
            auto at = [&](int f, int dx, int dy, int dz) -> double {
                return sp[(z + dz - pb) % NS][f][c0 + dy * WR + dx];
            };
            if constexpr (NF == 1) {
                const double f0 = c[0][c0];
                double acc = 0.0;
#pragma unroll
                for (int dz = -RZ; dz <= RZ; ++dz)
#pragma unroll
                    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                        for (int dx = -R; dx <= R; ++dx) {
                            const int sh = dx * dx + dy * dy + dz * dz;
                            const double w = iso_w(DIM, SCH, sh);
                            if (sh == 0 || w == 0.0) continue;
                            acc += w * (at(0, dx, dy, dz) - f0);
                        }
                st32(out, n, mu_bulk(f0, e) - e.kappa * (2.0 * acc));
            } else {
                double grx = 0.0, gry = 0.0, grz = 0.0, gmx = 0.0, gmy = 0.0, gmz = 0.0;
#pragma unroll
                for (int dz = -RZ; dz <= RZ; ++dz)
#pragma unroll
                    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                        for (int dx = -R; dx <= R; ++dx) {
                            const int sh = dx * dx + dy * dy + dz * dz;
                            const double w = iso_w(DIM, SCH, sh);
                            if (sh == 0 || w == 0.0) continue;
                            const double vr = w * at(0, dx, dy, dz), vm = w * at(1, dx, dy, dz);
                            if (dx) { grx += dx * vr; gmx += dx * vm; }
                            if (dy) { gry += dy * vr; gmy += dy * vm; }
                            if (dz) { grz += dz * vr; gmz += dz * vm; }
                        }
                const double r = c[0][c0];
                st32(out, n, -r * gmx + cs2 * grx);
                st32(out + N, n, -r * gmy + cs2 * gry);
                if constexpr (DIM == 3) st32(out + 2 * (size_t)N, n, -r * gmz + cs2 * grz);
            }
        } else if constexpr (NF == 1) {
            const double f0 = c[0][c0];
            double acc = DIM * d2(SCH, 0) * f0;
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                const double w = d2(SCH, m);
                acc += w * (c[0][c0 + m] + c[0][c0 - m]);
                acc += w * (c[0][c0 + m * WR] + c[0][c0 - m * WR]);
                if constexpr (DIM == 3) acc += w * (q[0][R + m] + q[0][R - m]);
            }
            if constexpr (DIM != 3) mb = mu_bulk(f0, e);
            // solid nodes (wetting boundary) carry the wall's chemical potential
            st32(out, n, g.wl && g.wl[n] ? e.mu_wall : mb - e.kappa * acc);
        } else {
            double grx = 0.0, gry = 0.0, grz = 0.0, gmx = 0.0, gmy = 0.0, gmz = 0.0;
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                const double w = d1(SCH, m);
                grx += w * (c[0][c0 + m] - c[0][c0 - m]);
                gry += w * (c[0][c0 + m * WR] - c[0][c0 - m * WR]);
                gmx += w * (c[1][c0 + m] - c[1][c0 - m]);
                gmy += w * (c[1][c0 + m * WR] - c[1][c0 - m * WR]);
                if constexpr (DIM == 3) {
                    grz += w * (q[0][R + m] - q[0][R - m]);
                    gmz += w * (q[1][R + m] - q[1][R - m]);
                }
            }
            const double r = c[0][c0];
            st32(out, n, -r * gmx + cs2 * grx);
            st32(out + N, n, -r * gmy + cs2 * gry);
            if constexpr (DIM == 3) st32(out + 2 * (size_t)N, n, -r * gmz + cs2 * grz);
        }
    }
}

template <int DIM, int SCH>
inline void launch_mu_march(const double* rho, double* mu, const Grid& g, const Eos& e, hipStream_t st)
{
    const TileGeom t = march_tiles(g, DIM == 3, MZ);
    const unsigned nb = (unsigned)(t.ntx * t.nty * t.nsz);
    hipLaunchKernelGGL((k_march<DIM, SCH, 1>), dim3(nb), dim3(MX * MY), 0, st, rho, nullptr, mu, g, t, e);
}

template <int DIM, int SCH>
inline void launch_force_march(const double* rho, const double* mu, double* F, const Grid& g, const Eos& e,
                               hipStream_t st)
{
    constexpr int TYM = DIM == 3 && !is_iso(SCH) ? 16 : MY;
    const TileGeom t = march_tiles(g, DIM == 3, 2 * MZ, TYM);
    const unsigned nb = (unsigned)(t.ntx * t.nty * t.nsz);
    hipLaunchKernelGGL((k_march<DIM, SCH, 2, TYM>), dim3(nb), dim3(MX * TYM), 0, st, rho, mu, F, g, t, e);
}

// ---------------------------------------------------------------------------
// k_mf: the chemical potential and the force of the explicit CD schemes in
// one z-march (3D).  mu_hat = k^2 psi'(rho) - kappa_hat lap(rho) (Eq 15, 16)
// never goes to memory: each workgroup computes it on its tile plus an R-wide
// ring and forms F = -rho grad(mu_hat) + cs^2 grad(rho) (Eq 12) for the tile,
// reading rho once and writing F.
// Per plane p of the march:
//   * rho of plane p is staged in LDS over the tile plus a 2R ring; every
//     mu_hat cell (tile + R) takes its value into a register queue (planes
//     p - 2R .. p) and its in-plane Laplacian terms into a second queue
//     (planes p - R .. p);
//   * mu_hat of plane p - R follows from the two queues and goes to an LDS
//     ring of R + 1 planes (in-plane arms of grad mu_hat); the thread's own
//     column also keeps it in a register queue (z arms);
//   * rho of plane p - 2R leaves the queues through LDS for the in-plane arms
//     of grad rho, and F of plane p - 2R is stored.
// The march starts 2R planes before its segment.  Each thread owns one tile
// node; the ring cells are dealt out as second cells to the first threads.
// ---------------------------------------------------------------------------
template <int SCH, int TY>
__global__ void __launch_bounds__(64 * TY, TY <= 8 ? 4 : 1)
k_mf(const double* __restrict__ rho, double* __restrict__ out, Grid g, TileGeom tg, Eos e)
{
    constexpr int R = radius(SCH);
    constexpr int NTH = 64 * TY;
    constexpr int WP = 64 + 4 * R, HP = TY + 4 * R, CP = WP * HP;   // staged rho: tile + 2R ring
    constexpr int WM = 64 + 2 * R, HM = TY + 2 * R, CM = WM * HM;   // mu_hat cells: tile + R ring
    constexpr int NH = CM - NTH;                                   // mu_hat cells outside the tile
    constexpr int SMC = 1 + (NH + NTH - 1) / NTH;                  // mu_hat cells per thread
    constexpr int SPP = (CP + NTH - 1) / NTH;                      // staged rho cells per thread
    constexpr int NSL = R + 1;                                     // mu_hat planes kept in LDS
    constexpr int QZ = 2 * R + 1;
    constexpr double cs2 = 1.0 / 3.0;
    __shared__ double sp[CP];
    __shared__ double sm[NSL][CM];
    __shared__ double sr[CM];

    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int nxy = (int)g.nxy;
    const unsigned N = (unsigned)g.N;
    int b = blockIdx.x;
    {
        const int nb = gridDim.x, per = nb / 8;
        if (b < per * 8) b = (b % 8) * per + b / 8;
    }
    const int tx = b % tg.ntx;
    const int ty = (b / tg.ntx) % tg.nty;
    const int sz = b / (tg.ntx * tg.nty);
    const int x0 = tx * 64, y0 = ty * TY;
    const int lid = threadIdx.x;
    const int lx = lid % 64, ly = lid / 64;
    const bool in = x0 + lx < nx && y0 + ly < ny;
    const int z0 = sz * tg.mz, z1 = min(z0 + tg.mz, nz);

    // in-plane offsets of the staged rho cells this thread loads
    unsigned off[SPP];
#pragma unroll
    for (int k = 0; k < SPP; ++k) {
        const int idx = lid + k * NTH;
        const int hy = idx / WP, hx = idx - hy * WP;
        off[k] = idx < CP ? (unsigned)(pwrap(y0 - 2 * R + hy, ny) * nx + pwrap(x0 - 2 * R + hx, nx)) : 0u;
    }
    // this thread's mu_hat cells: its own node, then ring cells h = lid,
    // lid + NTH, ... in the order top band, bottom band, side bands
    int cm[SMC], cq[SMC];
    bool cv[SMC];
#pragma unroll
    for (int s = 0; s < SMC; ++s) {
        int mr, mc;
        if (s == 0) {
            mr = ly + R; mc = lx + R;
            cv[s] = true;
        } else {
            const int h = (s - 1) * NTH + lid;
            cv[s] = h < NH;
            if (h < R * WM) { mr = h / WM; mc = h - mr * WM; }
            else if (h < 2 * R * WM) { const int h2 = h - R * WM; mr = HM - R + h2 / WM; mc = h2 % WM; }
            else {
                const int h3 = cv[s] ? h - 2 * R * WM : 0;
                const int c = h3 % (2 * R);
                mr = R + h3 / (2 * R);
                mc = c < R ? c : 64 + c;
            }
            if (!cv[s]) { mr = R; mc = R; }
        }
        cm[s] = mr * WM + mc;
        cq[s] = (mr + R) * WP + (mc + R);
    }

    double rq[SMC][QZ];     // rho of each cell, planes p - 2R .. p (index 0 the oldest)
    double lq[SMC][R + 1];  // in-plane Laplacian terms of each cell, planes p - R .. p
    double ro[R];           // own column, planes p - 3R .. p - 2R - 1 (rq[0] continued)
    double mq[QZ];          // own column mu_hat, planes p - 3R .. p - R
#pragma unroll
    for (int s = 0; s < SMC; ++s) {
#pragma unroll
        for (int k = 0; k < QZ; ++k) rq[s][k] = 0.0;
#pragma unroll
        for (int k = 0; k <= R; ++k) lq[s][k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) ro[k] = 0.0;
#pragma unroll
    for (int k = 0; k < QZ; ++k) mq[k] = 0.0;

    double sv[SPP];
    auto fetch = [&](int p) {
        const unsigned zo = (unsigned)(pwrap(p, nz) * nxy);
#pragma unroll
        for (int k = 0; k < SPP; ++k)
            if (lid + k * NTH < CP) sv[k] = ld32(rho, zo + off[k]);
    };
    const int pb = z0 - 2 * R, pe = z1 - 1 + 2 * R;
    fetch(pb);
    for (int p = pb; p <= pe; ++p) {
        // bulk potential of the mu_hat cells of plane p - R (rq[s][R + 1]
        // before the queues advance), evaluated before the barrier so that it
        // fills the wait for the other waves' stores
        double mb[SMC];
#pragma unroll
        for (int s = 0; s < SMC; ++s) mb[s] = 0.0;
        if (p >= z0) {
#pragma unroll
            for (int s = 0; s < SMC; ++s)
                if (cv[s]) mb[s] = mu_bulk(rq[s][R + 1], e);
        }
#pragma unroll
        for (int k = 0; k < SPP; ++k)
            if (lid + k * NTH < CP) sp[lid + k * NTH] = sv[k];
        __syncthreads();
        if (p < pe) fetch(p + 1);
        // queues advance by one plane; plane p enters
#pragma unroll
        for (int k = 0; k < R - 1; ++k) ro[k] = ro[k + 1];
        ro[R - 1] = rq[0][0];
#pragma unroll
        for (int s = 0; s < SMC; ++s) {
#pragma unroll
            for (int k = 0; k < QZ - 1; ++k) rq[s][k] = rq[s][k + 1];
#pragma unroll
            for (int k = 0; k < R; ++k) lq[s][k] = lq[s][k + 1];
            if (cv[s]) {
                const int o = cq[s];
                const double v = sp[o];
                double a = 2.0 * d2(SCH, 0) * v;
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    const double w = d2(SCH, m);
                    a += w * (sp[o + m] + sp[o - m]);
                    a += w * (sp[o + m * WP] + sp[o - m * WP]);
                }
                rq[s][QZ - 1] = v;
                lq[s][R] = a;
            }
        }
        // mu_hat of plane p - R (Eq 16)
        if (p >= z0) {
            double (*M)[CM] = sm + pwrap(p - R, NSL);
#pragma unroll
            for (int s = 0; s < SMC; ++s) {
                if (!cv[s]) continue;
                const double c = rq[s][R];
                double acc = lq[s][0] + d2(SCH, 0) * c;
#pragma unroll
                for (int m = 1; m <= R; ++m) acc += d2(SCH, m) * (rq[s][R + m] + rq[s][R - m]);
                const double mu = mb[s] - e.kappa * acc;
                (*M)[cm[s]] = mu;
                if (s == 0) {
#pragma unroll
                    for (int k = 0; k < QZ - 1; ++k) mq[k] = mq[k + 1];
                    mq[QZ - 1] = mu;
                }
            }
        }
        // rho of plane p - 2R for the in-plane arms of grad rho
        const int z = p - 2 * R;
        if (z >= z0) {
#pragma unroll
            for (int s = 0; s < SMC; ++s)
                if (cv[s]) sr[cm[s]] = rq[s][0];
        }
        __syncthreads();
        // F of plane z (Eq 12)
        if (z >= z0 && in) {
            const double* M = sm[pwrap(z, NSL)];
            const int o = cm[0];
            double grx = 0.0, gry = 0.0, grz = 0.0, gmx = 0.0, gmy = 0.0, gmz = 0.0;
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                const double w = d1(SCH, m);
                grx += w * (sr[o + m] - sr[o - m]);
                gry += w * (sr[o + m * WM] - sr[o - m * WM]);
                gmx += w * (M[o + m] - M[o - m]);
                gmy += w * (M[o + m * WM] - M[o - m * WM]);
                grz += w * (rq[0][m] - ro[R - m]);
                gmz += w * (mq[R + m] - mq[R - m]);
            }
            const double r = rq[0][0];
            const unsigned n = (unsigned)(z * nxy + (y0 + ly) * nx + x0 + lx);
            st32(out, n, -r * gmx + cs2 * grx);
            st32(out + N, n, -r * gmy + cs2 * gry);
            st32(out + 2 * (size_t)N, n, -r * gmz + cs2 * grz);
        }
    }
}

// Segment length of the k_mf march: the 2R planes it reads before its
// segment are a smaller share of a long one.
constexpr int kMfZ = 64;

template <int SCH>
inline void launch_mf(int ty, const double* rho, double* F, const Grid& g, const Eos& e, hipStream_t st)
{
    TileGeom t;
    t.ntx = (g.nx + 63) / 64;
    t.nty = (g.ny + ty - 1) / ty;
    t.mz = kMfZ;
    t.nsz = (g.nz + kMfZ - 1) / kMfZ;
    const unsigned nb = (unsigned)(t.ntx * t.nty * t.nsz);
    if (ty == 16) hipLaunchKernelGGL((k_mf<SCH, 16>), dim3(nb), dim3(64 * 16), 0, st, rho, F, g, t, e);
    else hipLaunchKernelGGL((k_mf<SCH, 8>), dim3(nb), dim3(64 * 8), 0, st, rho, F, g, t, e);
}

// ---------------------------------------------------------------------------
// Collision of one node (Eq 1 SRT or D2Q9 MRT, Eq 6, Eq 8) from its pulled
// populations and force; each post-collision value goes to emit(i, o) as soon
// as it is formed.  FULL: SRT with tau = 1, where f* = feq(rho, u + du).
// ---------------------------------------------------------------------------
template <int LAT, bool FULL, typename Emit>
__device__ __forceinline__ void collide_emit(const double (&f)[Lat<LAT>::Q], double Fx, double Fy, double Fz,
                                             const Relax& rx, Emit&& emit)
{
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        jx += L::ex(i) * f[i]; jy += L::ey(i) * f[i]; jz += L::ez(i) * f[i];
    }
    const double ir = 1.0 / r;
    const double ux = jx * ir, uy = jy * ir, uz = jz * ir;
    const double vx = ux + Fx * ir, vy = uy + Fy * ir, vz = uz + Fz * ir;
    const double uu = 1.0 - 1.5 * (ux * ux + uy * uy + uz * uz);
    const double vv = 1.0 - 1.5 * (vx * vx + vy * vy + vz * vz);
    double om[LAT == 0 ? 9 : 1];   // MRT post-collision values (D2Q9)
    if constexpr (LAT == 0 && !FULL) {
        if (rx.mrt) {
            double fe[9], fv[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const double wr = L::w(i) * r;
                const double eu = L::ex(i) * ux + L::ey(i) * uy;
                const double ev = L::ex(i) * vx + L::ey(i) * vy;
                fe[i] = wr * (uu + eu * (3.0 + 4.5 * eu));
                fv[i] = wr * (vv + ev * (3.0 + 4.5 * ev));
            }
            mrt_post(f, fe, fv, rx, om);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double wr = L::w(i) * r;
        const double ev = L::ex(i) * vx + L::ey(i) * vy + L::ez(i) * vz;
        const double fv = wr * (vv + ev * (3.0 + 4.5 * ev));
        double o = fv;
        if constexpr (!FULL) {
            const double eu = L::ex(i) * ux + L::ey(i) * uy + L::ez(i) * uz;
            const double fe = wr * (uu + eu * (3.0 + 4.5 * eu));
            o = fv + rx.omo * (f[i] - fe);
            if constexpr (LAT == 0) {
                if (rx.mrt) o = om[i];
            }
        }
        emit(i, o);
    }
}

// ---------------------------------------------------------------------------
// Ring collide with a precomputed force: the same tile + ring scheme as
// k_fused, but the force field comes from k_march (three loads per node), so
// the kernel holds no stencil state.  The next plane's pulls are issued right
// after the gather of the current plane, overlapping the second barrier.
// ---------------------------------------------------------------------------
template <int LAT, int TX, int TY, int OCC, bool PF, bool FULL>
__global__ void __launch_bounds__((TX + 2) * (TY + 2), OCC)
k_ring(const double* __restrict__ S, double* __restrict__ Sn, const double* __restrict__ F,
       double* __restrict__ rho_next, Grid g, TileGeom tg, Relax rx)
{
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    constexpr int W = TX + 2, H = TY + 2, NTH = W * H;
    constexpr int NCL = LAT == 1 ? 16 : 8;
    __shared__ double xs[NCL][NTH];

    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int nxy = (int)g.nxy, N = (int)g.N;
    int b = blockIdx.x;
    {
        const int nb = gridDim.x, per = nb / 8;
        if (b < per * 8) b = (b % 8) * per + b / 8;
    }
    const int tx = b % tg.ntx;
    const int ty = (b / tg.ntx) % tg.nty;
    const int sz = b / (tg.ntx * tg.nty);
    const int x0 = tx * TX, y0 = ty * TY;
    const int wx = min(TX, nx - x0), wy = min(TY, ny - y0);
    // Tile nodes first, one row of TX per TX lanes (rows start on wave
    // boundaries when TX = 64, so the tile's loads and stores are aligned),
    // then the ring: bottom row, top row, left column, right column.
    const int lid = threadIdx.x;
    int lx, ly;
    if (lid < TX * TY) {
        lx = 1 + lid % TX; ly = 1 + lid / TX;
    } else {
        const int r = lid - TX * TY;
        if (r < W) { lx = r; ly = 0; }
        else if (r < 2 * W) { lx = r - W; ly = H - 1; }
        else if (r < 2 * W + TY) { lx = 0; ly = 1 + r - 2 * W; }
        else { lx = W - 1; ly = 1 + r - 2 * W - TY; }
    }
    const int slot = ly * W + lx;   // LDS exchange position
    const bool active = lx <= wx + 1 && ly <= wy + 1;
    const bool inner = lx >= 1 && lx <= wx && ly >= 1 && ly <= wy;
    const int x = active ? wrapc(x0 - 1 + lx, nx) : 0;
    const int y = active ? wrapc(y0 - 1 + ly, ny) : 0;
    const int xm = wrapc(x - 1, nx), xp = wrapc(x + 1, nx);
    const int yc = y * nx, ym = wrapc(y - 1, ny) * nx, yp = wrapc(y + 1, ny) * nx;
    const int z0 = LAT == 1 ? sz * FZ : 0;
    const int z1 = LAT == 1 ? min(z0 + FZ, nz) : 1;

    double f[Q], Fx = 0.0, Fy = 0.0, Fz = 0.0;
    double fn[PF ? Q : 1], Fxn = 0.0, Fyn = 0.0, Fzn = 0.0;
    auto pull_plane = [&](int z, double (&f)[Q], double& Fx, double& Fy, double& Fz) {
        const int zo = z * nxy;
        const int zmo = LAT == 1 ? wrapc(z - 1, nz) * nxy : 0;
        const int zpo = LAT == 1 ? wrapc(z + 1, nz) * nxy : 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int ox = L::ex(i) == 1 ? xm : L::ex(i) == -1 ? xp : x;
            const int oy = L::ey(i) == 1 ? ym : L::ey(i) == -1 ? yp : yc;
            const int oz = L::ez(i) == 1 ? zmo : L::ez(i) == -1 ? zpo : zo;
            f[i] = ld32(S + (long long)i * g.ps, (unsigned)(oz + oy + ox));
        }
        const unsigned n = (unsigned)(zo + yc + x);
        Fx = ld32(F, n);
        Fy = ld32(F + N, n);
        if constexpr (LAT == 1) Fz = ld32(F + 2LL * N, n);
    };

    double acc_m1 = 0.0, acc_0 = 0.0;
    const int zb = LAT == 1 ? z0 - 1 : 0, ze = LAT == 1 ? z1 : 0;
    if (active) pull_plane(LAT == 1 ? pwrap(zb, nz) : 0, f, Fx, Fy, Fz);
    for (int zr = zb; zr <= ze; ++zr) {
        const int z = LAT == 1 ? pwrap(zr, nz) : 0;
        // PF: the next plane's loads go out a whole plane ahead (registers
        // double-buffered); otherwise they are issued after the gather
        if constexpr (PF) {
            if (active && zr < ze) pull_plane(pwrap(zr + 1, nz), fn, Fxn, Fyn, Fzn);
        }
        double own_m1 = 0.0, own_0 = 0.0, own_p1 = 0.0;   // post-collision values without in-plane shift
        if (active) {
            const bool store = inner && zr >= z0 && zr < z1;
            const int n = z * nxy + yc + x;
            collide_emit<LAT, FULL>(f, Fx, Fy, Fz, rx, [&](int i, double o) {
                if (store) st32(Sn + (long long)i * g.ps, (unsigned)n, o);
                if (xcls_of<LAT>(i) >= 0) xs[xcls_of<LAT>(i)][slot] = o;
                else if (L::ez(i) == -1) own_m1 = o;
                else if (L::ez(i) == 0) own_0 = o;
                else own_p1 = o;
            });
        }
        __syncthreads();
        double a_m1 = own_m1, a_0 = own_0, a_p1 = own_p1;
        if (inner) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (xcls_of<LAT>(i) < 0) continue;
                const double v = xs[xcls_of<LAT>(i)][(ly - L::ey(i)) * W + (lx - L::ex(i))];
                if (L::ez(i) == -1) a_m1 += v; else if (L::ez(i) == 0) a_0 += v; else a_p1 += v;
            }
        }
        if constexpr (!PF) {
            if (active && zr < ze) pull_plane(pwrap(zr + 1, nz), f, Fx, Fy, Fz);
        }
        __syncthreads();
        if (inner) {
            if constexpr (LAT == 1) {
                acc_m1 += a_m1;
                if (zr - 1 >= z0 && zr - 1 < z1) st32(rho_next, (unsigned)((zr - 1) * nxy + yc + x), acc_m1);
                acc_m1 = acc_0 + a_0;
                acc_0 = a_p1;
            } else {
                rho_next[yc + x] = a_0;
            }
        }
        if constexpr (PF) {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = fn[i];
            Fx = Fxn; Fy = Fyn; Fz = Fzn;
        }
    }
}

// ---------------------------------------------------------------------------
// Tile collide without the ring, for grids tiled exactly by 64 x TY tiles.
// Every node of the tile is collided once.  Values that stay inside the tile
// reach their destination through LDS and give the tile's partial rho(t+1);
// the first NR lanes also sum, for each ring cell around the tile, the values
// that leave the tile into it, and store those sums.  k_fix then adds, at
// every node on a tile edge, the sums the neighbouring tiles left for it.  In
// z the segment is marched with one extra plane at each end, as in k_ring.
// ---------------------------------------------------------------------------
template <int TY>
struct TileRing {
    static constexpr int NR = 132 + 2 * TY;           // ring cells of a 64 x TY tile
    static constexpr int NB = 2 * 64 + 2 * (TY - 2);  // edge nodes of the tile
    // ring cell k -> (rx, ry) relative to the tile origin
    __host__ __device__ static void cell(int k, int& rx, int& ry)
    {
        if (k < 66) { rx = k - 1; ry = -1; }
        else if (k < 132) { rx = k - 67; ry = TY; }
        else if (k < 132 + TY) { rx = -1; ry = k - 132; }
        else { rx = 64; ry = k - 132 - TY; }
    }
    // (rx, ry) -> k, or -1 if it is no ring cell
    __host__ __device__ static int index(int rx, int ry)
    {
        if (rx < -1 || rx > 64 || ry < -1 || ry > TY) return -1;
        if (ry == -1) return rx + 1;
        if (ry == TY) return rx + 67;
        if (rx == -1) return 132 + ry;
        if (rx == 64) return 132 + TY + ry;
        return -1;
    }
};

inline bool tile_fits(const Grid& g, int ty) { return g.nx % 64 == 0 && g.ny % ty == 0; }

// WALL: the wetting boundary, from the per-node mask wb (bit i: x - e_i is
// solid; bit 31: the node is solid).  A fluid node pulls, for each direction
// whose source is solid, its own post-collision value of the opposite
// direction (halfway bounce-back), and adds those same values to its
// rho(t+1); solid nodes do not collide and send nothing.
// ZR (3D, no walls): a segment marches its own planes only.  What its first
// plane sends down (into the last plane of the segment below) and what its last
// plane sends up go to zring, slots 0 and 1 of the tile (NTH in-tile values,
// then NR ring cells), and k_fix_zr adds them, instead of every segment
// pulling and colliding one extra plane at each end.
template <int LAT, int TY, bool FULL, bool WALL = false, bool ZR = false>
__global__ void __launch_bounds__(64 * TY, TY <= 8 ? 2 : 1)
k_tile(const double* __restrict__ S, double* __restrict__ Sn, const double* __restrict__ F,
       double* __restrict__ rho_next, double* __restrict__ ringsum, Grid g, TileGeom tg, Relax rx,
       const unsigned* __restrict__ wb = nullptr, double* __restrict__ zring = nullptr)
{
    static_assert(!ZR || (LAT == 1 && !WALL), "z-ring segments are for the 3D collide without walls");
    using L = Lat<LAT>;
    using TR = TileRing<TY>;
    constexpr int Q = L::Q;
    constexpr int NTH = 64 * TY;
    constexpr int NCL = LAT == 1 ? 16 : 8;
    __shared__ double xs[NCL][NTH];

    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int nxy = (int)g.nxy, N = (int)g.N;
    int b = blockIdx.x;
    {
        const int nb = gridDim.x, per = nb / 8;
        if (b < per * 8) b = (b % 8) * per + b / 8;
    }
    const int tx = b % tg.ntx;
    const int ty = (b / tg.ntx) % tg.nty;
    const int sz = b / (tg.ntx * tg.nty);
    const int lid = threadIdx.x;
    const int lx = lid % 64, ly = lid / 64;
    const int x = tx * 64 + lx, y = ty * TY + ly;
    const int xm = wrapc(x - 1, nx), xp = wrapc(x + 1, nx);
    const int yc = y * nx, ym = wrapc(y - 1, ny) * nx, yp = wrapc(y + 1, ny) * nx;
    const int z0 = LAT == 1 ? sz * tg.mz : 0;
    const int z1 = LAT == 1 ? min(z0 + tg.mz, nz) : 1;
    const int MZT = LAT == 1 ? tg.mz : 1;   // ring-sum planes per segment
    double* rs = ringsum + (size_t)b * MZT * TR::NR;
    const bool ring = lid < TR::NR;
    int rcx = 0, rcy = 0;
    if (ring) TR::cell(lid, rcx, rcy);

    double f[Q], Fx = 0.0, Fy = 0.0, Fz = 0.0;
    unsigned bits = 0, bits_next = 0;   // wall mask of the plane pulled last / next
    auto pull_plane = [&](int z) {
        const int zo = z * nxy;
        const int zmo = LAT == 1 ? wrapc(z - 1, nz) * nxy : 0;
        const int zpo = LAT == 1 ? wrapc(z + 1, nz) * nxy : 0;
        const unsigned n = (unsigned)(zo + yc + x);
        if constexpr (WALL) bits = bits_next;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int ox = L::ex(i) == 1 ? xm : L::ex(i) == -1 ? xp : x;
            const int oy = L::ey(i) == 1 ? ym : L::ey(i) == -1 ? yp : yc;
            const int oz = L::ez(i) == 1 ? zmo : L::ez(i) == -1 ? zpo : zo;
            if constexpr (WALL) {
                const bool bb = (bits >> i) & 1u;
                f[i] = ld32(S + (long long)(bb ? L::opp(i) : i) * g.ps, bb ? n : (unsigned)(oz + oy + ox));
            } else {
                f[i] = ld32(S + (long long)i * g.ps, (unsigned)(oz + oy + ox));
            }
        }
        Fx = ld32(F, n);
        Fy = ld32(F + N, n);
        if constexpr (LAT == 1) Fz = ld32(F + 2LL * N, n);
    };

    double acc_m1 = 0.0, acc_0 = 0.0, racc_m1 = 0.0, racc_0 = 0.0;
    const int zb = LAT == 1 ? (ZR ? z0 : z0 - 1) : 0, ze = LAT == 1 ? (ZR ? z1 - 1 : z1) : 0;
    // the mask is loaded one plane ahead of the pulls it steers
    if constexpr (WALL) bits_next = wb[(LAT == 1 ? pwrap(zb, nz) : 0) * nxy + yc + x];
    pull_plane(LAT == 1 ? pwrap(zb, nz) : 0);
    if constexpr (WALL) {
        if (LAT == 1 && zb < ze) bits_next = wb[pwrap(zb + 1, nz) * nxy + yc + x];
    }
    for (int zr = zb; zr <= ze; ++zr) {
        const int z = LAT == 1 ? pwrap(zr, nz) : 0;
        double own_m1 = 0.0, own_0 = 0.0, own_p1 = 0.0;
        double ob[WALL ? Q : 1];   // this node's post-collision values (bounce-back)
        const unsigned mb = bits;
        const bool solid = WALL && (mb >> 31);
        {
            const bool store = zr >= z0 && zr < z1;
            const int n = z * nxy + yc + x;
            if (!solid) {
                collide_emit<LAT, FULL>(f, Fx, Fy, Fz, rx, [&](int i, double o) {
                    if (store) st32(Sn + (long long)i * g.ps, (unsigned)n, o);
                    if (xcls_of<LAT>(i) >= 0) xs[xcls_of<LAT>(i)][lid] = o;
                    else if (L::ez(i) == -1) own_m1 = o;
                    else if (L::ez(i) == 0) own_0 = o;
                    else own_p1 = o;
                    if constexpr (WALL) ob[i] = o;
                });
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    if (xcls_of<LAT>(i) >= 0) xs[xcls_of<LAT>(i)][lid] = 0.0;
                    if constexpr (WALL) ob[i] = 0.0;
                }
            }
        }
        __syncthreads();
        // values arriving from inside the tile, at the own node and (first NR
        // lanes) at one ring cell
        double a_m1 = own_m1, a_0 = own_0, a_p1 = own_p1, r_m1 = 0.0, r_0 = 0.0, r_p1 = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (xcls_of<LAT>(i) < 0) continue;
            const int sx = lx - L::ex(i), sy = ly - L::ey(i);
            if (sx >= 0 && sx < 64 && sy >= 0 && sy < TY) {
                const double v = xs[xcls_of<LAT>(i)][sy * 64 + sx];
                if (L::ez(i) == -1) a_m1 += v; else if (L::ez(i) == 0) a_0 += v; else a_p1 += v;
            }
            if (ring) {
                const int qx = rcx - L::ex(i), qy = rcy - L::ey(i);
                if (qx >= 0 && qx < 64 && qy >= 0 && qy < TY) {
                    const double v = xs[xcls_of<LAT>(i)][qy * 64 + qx];
                    if (L::ez(i) == -1) r_m1 += v; else if (L::ez(i) == 0) r_0 += v; else r_p1 += v;
                }
            }
        }
        if constexpr (WALL) {
            // values sent towards solid neighbours come back to this node
            if (!solid) {
#pragma unroll
                for (int j = 1; j < Q; ++j)
                    if ((mb >> j) & 1u) a_0 += ob[L::opp(j)];
            }
        }
        if (zr < ze) pull_plane(pwrap(zr + 1, nz));
        if constexpr (WALL) {
            if (LAT == 1 && zr + 1 < ze) bits_next = wb[pwrap(zr + 2, nz) * nxy + yc + x];
        }
        __syncthreads();
        if constexpr (LAT == 1) {
            acc_m1 += a_m1;
            racc_m1 += r_m1;
            if (zr - 1 >= z0 && zr - 1 < z1) {
                st32(rho_next, (unsigned)((zr - 1) * nxy + yc + x), acc_m1);
                if (ring) rs[(zr - 1 - z0) * TR::NR + lid] = racc_m1;
            } else if (ZR && zr == zb) {
                // what the first plane sends into the last plane of the segment below
                double* zd = zring + (size_t)b * 2 * (NTH + TR::NR);
                zd[lid] = acc_m1;
                if (ring) zd[NTH + lid] = racc_m1;
            }
            acc_m1 = acc_0 + a_0;
            acc_0 = a_p1;
            racc_m1 = racc_0 + r_0;
            racc_0 = r_p1;
        } else {
            rho_next[yc + x] = a_0;
            if (ring) rs[lid] = r_0;
        }
    }
    if constexpr (ZR) {
        // what the last plane sends into the first plane of the segment above,
        // and the last plane itself without what that plane sends down
        double* zu = zring + ((size_t)b * 2 + 1) * (NTH + TR::NR);
        zu[lid] = acc_0;
        if (ring) zu[NTH + lid] = racc_0;
        st32(rho_next, (unsigned)(ze * nxy + yc + x), acc_m1);
        if (ring) rs[(ze - z0) * TR::NR + lid] = racc_m1;
    }
}

// Adds to every node on a tile edge the ring sums the (up to eight)
// neighbouring tiles left for it, in a fixed order.
template <int TY>
__global__ void __launch_bounds__(256) k_fix(double* __restrict__ rho_next, const double* __restrict__ ringsum,
                                            Grid g, TileGeom tg, int mzt)
{
    using TR = TileRing<TY>;
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int ntile = tg.ntx * tg.nty * tg.nsz;
    if (t >= ntile * mzt * TR::NB) return;
    const int e = t % TR::NB;
    const int rest = t / TR::NB;
    const int zl = rest % mzt;
    const int tile = rest / mzt;
    const int tx = tile % tg.ntx, ty = (tile / tg.ntx) % tg.nty, sz = tile / (tg.ntx * tg.nty);
    const int z = sz * mzt + zl;
    if (z >= g.nz) return;
    int lx, ly;
    if (e < 64) { lx = e; ly = 0; }
    else if (e < 128) { lx = e - 64; ly = TY - 1; }
    else if (e < 128 + TY - 2) { lx = 0; ly = 1 + e - 128; }
    else { lx = 63; ly = 1 + e - 128 - (TY - 2); }
    const unsigned n = (unsigned)(z * (int)g.nxy + (ty * TY + ly) * g.nx + tx * 64 + lx);
    // neighbouring tiles, wrapped without divisions
    const int txs[3] = { tx == 0 ? tg.ntx - 1 : tx - 1, tx, tx + 1 == tg.ntx ? 0 : tx + 1 };
    const int tys[3] = { ty == 0 ? tg.nty - 1 : ty - 1, ty, ty + 1 == tg.nty ? 0 : ty + 1 };
    double acc = ld32(rho_next, n);
#pragma unroll
    for (int dty = -1; dty <= 1; ++dty)
#pragma unroll
        for (int dtx = -1; dtx <= 1; ++dtx) {
            if (dtx == 0 && dty == 0) continue;
            const int k = TR::index(lx - 64 * dtx, ly - TY * dty);
            if (k < 0) continue;
            const int tn = (sz * tg.nty + tys[dty + 1]) * tg.ntx + txs[dtx + 1];
            acc += ringsum[((size_t)tn * mzt + zl) * TR::NR + k];
        }
    st32(rho_next, n, acc);
}

// The fix of the z-ring segments: per tile segment, every node of its first
// and last plane, and the edge nodes of the planes between.  A node adds, in
// this order, the ring sums the neighbouring tiles of its segment left for it
// (edge nodes), then on the first plane what the segment below sent up (its own
// tile's in-tile value, then the neighbouring tiles' ring cells), then on the
// last plane what the segment above sent down (the same way).
template <int TY>
__global__ void __launch_bounds__(256) k_fix_zr(double* __restrict__ rho_next, const double* __restrict__ ringsum,
                                               const double* __restrict__ zring, Grid g, TileGeom tg, int mzt)
{
    using TR = TileRing<TY>;
    constexpr int NTH = 64 * TY, ZW = NTH + TR::NR;
    // one row of the grid per tile segment, its items along x
    const int per = 2 * NTH + (mzt - 2) * TR::NB;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= per) return;
    const int tile = blockIdx.y;
    const int tx = tile % tg.ntx, ty = (tile / tg.ntx) % tg.nty, sz = tile / (tg.ntx * tg.nty);
    const int z0 = sz * mzt, planes = min(mzt, g.nz - z0);
    int zl, lx, ly;
    if (j < 2 * NTH) {
        const int which = j / NTH, lid = j - which * NTH;
        if (which == 1 && planes == 1) return;   // one plane: the first-plane item takes both ends
        zl = which == 0 ? 0 : planes - 1;
        lx = lid % 64;
        ly = lid / 64;
    } else {
        const int i = j - 2 * NTH;
        zl = 1 + i / TR::NB;
        if (zl >= planes - 1) return;
        const int e = i % TR::NB;
        if (e < 64) { lx = e; ly = 0; }
        else if (e < 128) { lx = e - 64; ly = TY - 1; }
        else if (e < 128 + TY - 2) { lx = 0; ly = 1 + e - 128; }
        else { lx = 63; ly = 1 + e - 128 - (TY - 2); }
    }
    const bool edge = lx == 0 || lx == 63 || ly == 0 || ly == TY - 1;
    const unsigned n = (unsigned)((z0 + zl) * (int)g.nxy + (ty * TY + ly) * g.nx + tx * 64 + lx);
    const int txs[3] = { tx == 0 ? tg.ntx - 1 : tx - 1, tx, tx + 1 == tg.ntx ? 0 : tx + 1 };
    const int tys[3] = { ty == 0 ? tg.nty - 1 : ty - 1, ty, ty + 1 == tg.nty ? 0 : ty + 1 };
    double acc = ld32(rho_next, n);
    if (edge) {
#pragma unroll
        for (int dty = -1; dty <= 1; ++dty)
#pragma unroll
            for (int dtx = -1; dtx <= 1; ++dtx) {
                if (dtx == 0 && dty == 0) continue;
                const int k = TR::index(lx - 64 * dtx, ly - TY * dty);
                if (k < 0) continue;
                const int tn = (sz * tg.nty + tys[dty + 1]) * tg.ntx + txs[dtx + 1];
                acc += ringsum[((size_t)tn * mzt + zl) * TR::NR + k];
            }
    }
    // slot 1 of the segment below (first plane), slot 0 of the segment above (last plane)
#pragma unroll
    for (int end = 0; end < 2; ++end) {
        if (end == 0 ? zl != 0 : zl != planes - 1) continue;
        const int so = end == 0 ? (sz == 0 ? tg.nsz - 1 : sz - 1) : (sz + 1 == tg.nsz ? 0 : sz + 1);
        const int slot = end == 0 ? 1 : 0;
        acc += zring[((size_t)((so * tg.nty + ty) * tg.ntx + tx) * 2 + slot) * ZW + ly * 64 + lx];
        if (edge) {
#pragma unroll
            for (int dty = -1; dty <= 1; ++dty)
#pragma unroll
                for (int dtx = -1; dtx <= 1; ++dtx) {
                    if (dtx == 0 && dty == 0) continue;
                    const int k = TR::index(lx - 64 * dtx, ly - TY * dty);
                    if (k < 0) continue;
                    const int tn = (so * tg.nty + tys[dty + 1]) * tg.ntx + txs[dtx + 1];
                    acc += zring[((size_t)tn * 2 + slot) * ZW + NTH + k];
                }
        }
    }
    st32(rho_next, n, acc);
}

// Launch variants of the tile collide: tile height, z planes per segment, and
// whether the chemical potential and the force come from one march (k_mf) or
// from the two marches (k_march).  The taller tile halves the edge share (16%
// of the nodes instead of 29%) at one 1024-thread workgroup per CU; the longer
// segment halves the two planes each segment pulls beyond its own.  The ring-
// sum buffer has one slot per ring cell and plane of the lowest tile, for the
// planes of the longest segment.
// zr: z-ring segments (3D without walls; 64x16 tiles): no plane is pulled
// or collided twice, the segment ends are completed by k_fix_zr.
struct TileVariant { int ty, fz, mf, zr; };
constexpr TileVariant kTileVariants[] = { {8, 32, 0, 0}, {16, 32, 0, 0}, {8, 64, 0, 0}, {16, 64, 0, 0},
                                          {16, 32, 1, 0}, {16, 64, 1, 0}, {8, 64, 1, 0},
                                          {16, 32, 0, 1}, {16, 64, 0, 1}, {16, 64, 1, 1} };
constexpr int kNumTileVariants = 10;
constexpr int kZringTY = 16;
constexpr int kZringMinFZ = 32;
constexpr int kTileTY = 8;
constexpr int kTileMaxFZ = 64;

inline size_t ringsum_doubles(const Grid& g, bool three_d)
{
    const size_t ntile = (size_t)(g.nx / 64) * (g.ny / kTileTY);
    const size_t planes = three_d ? (size_t)((g.nz + kTileMaxFZ - 1) / kTileMaxFZ) * kTileMaxFZ : 1;
    return ntile * planes * TileRing<kTileTY>::NR;
}

// Doubles of the z-ring buffer: two slots of 64*16 in-tile values and the
// ring cells per tile segment, for the shortest z-ring segment.
inline size_t zring_doubles(const Grid& g)
{
    const size_t ntile = (size_t)(g.nx / 64) * (g.ny / kZringTY) * ((g.nz + kZringMinFZ - 1) / kZringMinFZ);
    return ntile * 2 * (64 * kZringTY + TileRing<kZringTY>::NR);
}

inline TileGeom tile_geom(const Grid& g, bool three_d, int ty, int fz)
{
    TileGeom t;
    t.ntx = g.nx / 64;
    t.nty = g.ny / ty;
    t.nsz = three_d ? (g.nz + fz - 1) / fz : 1;
    t.mz = three_d ? fz : 1;
    return t;
}

template <int LAT, int TY>
inline void launch_tile_ty(const double* S, double* Sn, const double* F, double* rho_next, double* ringsum,
                           const Grid& g, const Relax& rx, int fz, hipStream_t st, const unsigned* wb,
                           double* zring = nullptr)
{
    const TileGeom t = tile_geom(g, LAT == 1, TY, fz);
    const unsigned nb = (unsigned)(t.ntx * t.nty * t.nsz);
    const bool full = rx.omo == 0.0 && !rx.mrt;
    if constexpr (LAT == 1 && TY == kZringTY) {
        if (zring) {
            if (full)
                hipLaunchKernelGGL((k_tile<LAT, TY, true, false, true>), dim3(nb), dim3(64 * TY), 0, st, S, Sn, F,
                                   rho_next, ringsum, g, t, rx, nullptr, zring);
            else
                hipLaunchKernelGGL((k_tile<LAT, TY, false, false, true>), dim3(nb), dim3(64 * TY), 0, st, S, Sn, F,
                                   rho_next, ringsum, g, t, rx, nullptr, zring);
            return;
        }
    }
    if (wb) {
        if (full)
            hipLaunchKernelGGL((k_tile<LAT, TY, true, true>), dim3(nb), dim3(64 * TY), 0, st, S, Sn, F, rho_next,
                               ringsum, g, t, rx, wb);
        else
            hipLaunchKernelGGL((k_tile<LAT, TY, false, true>), dim3(nb), dim3(64 * TY), 0, st, S, Sn, F, rho_next,
                               ringsum, g, t, rx, wb);
    } else if (full) {
        hipLaunchKernelGGL((k_tile<LAT, TY, true>), dim3(nb), dim3(64 * TY), 0, st, S, Sn, F, rho_next, ringsum,
                           g, t, rx, nullptr);
    } else {
        hipLaunchKernelGGL((k_tile<LAT, TY, false>), dim3(nb), dim3(64 * TY), 0, st, S, Sn, F, rho_next, ringsum,
                           g, t, rx, nullptr);
    }
}

template <int TY>
inline void launch_fix_ty(double* rho_next, const double* ringsum, const Grid& g, bool three_d, int fz,
                          hipStream_t st, const double* zring = nullptr)
{
    const TileGeom t = tile_geom(g, three_d, TY, fz);
    if (zring) {
        const int per = 2 * 64 * TY + (t.mz - 2) * TileRing<TY>::NB;
        hipLaunchKernelGGL((k_fix_zr<TY>), dim3((unsigned)((per + 255) / 256), (unsigned)(t.ntx * t.nty * t.nsz)),
                           dim3(256), 0, st, rho_next, ringsum, zring, g, t, t.mz);
        return;
    }
    const long long items = (long long)t.ntx * t.nty * t.nsz * t.mz * TileRing<TY>::NB;
    hipLaunchKernelGGL((k_fix<TY>), dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, rho_next, ringsum,
                       g, t, t.mz);
}

// zring: the z-ring buffer, used by the variants with zr set (64x16 tiles, 3D).
template <int LAT>
inline void launch_tile(const TileVariant& v, const double* S, double* Sn, const double* F, double* rho_next,
                        double* ringsum, const Grid& g, const Relax& rx, hipStream_t st,
                        const unsigned* wb = nullptr, double* zring = nullptr)
{
    double* zr = v.zr ? zring : nullptr;
    if (v.ty == 16) launch_tile_ty<LAT, 16>(S, Sn, F, rho_next, ringsum, g, rx, v.fz, st, wb, zr);
    else launch_tile_ty<LAT, 8>(S, Sn, F, rho_next, ringsum, g, rx, v.fz, st, wb);
}

template <int LAT>
inline void launch_fix(const TileVariant& v, double* rho_next, const double* ringsum, const Grid& g, hipStream_t st,
                       const double* zring = nullptr)
{
    const double* zr = v.zr ? zring : nullptr;
    if (v.ty == 16) launch_fix_ty<16>(rho_next, ringsum, g, LAT == 1, v.fz, st, zr);
    else launch_fix_ty<8>(rho_next, ringsum, g, LAT == 1, v.fz, st);
}

struct RingVariant { int tx, ty, occ, pf; };
constexpr RingVariant kRingVariants[] = { {64, 8, 3, 0}, {64, 13, 2, 0}, {64, 8, 3, 1} };
constexpr int kNumRingVariants = 3;

inline TileGeom ring_tiles(int tx, int ty, const Grid& g, bool three_d)
{
    TileGeom t;
    t.ntx = (g.nx + tx - 1) / tx;
    t.nty = (g.ny + ty - 1) / ty;
    t.nsz = three_d ? (g.nz + FZ - 1) / FZ : 1;
    t.mz = FZ;
    return t;
}

template <int LAT, int TX, int TY, int OCC, bool PF>
inline void launch_ring_v(const double* S, double* Sn, const double* F, double* rho_next, const Grid& g,
                          const Relax& rx, hipStream_t st)
{
    const TileGeom t = ring_tiles(TX, TY, g, LAT == 1);
    const unsigned nb = (unsigned)(t.ntx * t.nty * t.nsz);
    if (rx.omo == 0.0 && !rx.mrt)
        hipLaunchKernelGGL((k_ring<LAT, TX, TY, OCC, PF, true>), dim3(nb), dim3((TX + 2) * (TY + 2)), 0, st, S, Sn, F,
                           rho_next, g, t, rx);
    else
        hipLaunchKernelGGL((k_ring<LAT, TX, TY, OCC, PF, false>), dim3(nb), dim3((TX + 2) * (TY + 2)), 0, st, S, Sn, F,
                           rho_next, g, t, rx);
}

template <int LAT>
inline void launch_ring_collide(int variant, const double* S, double* Sn, const double* F, double* rho_next,
                                const Grid& g, const Relax& rx, hipStream_t st)
{
    switch (variant) {
    case 1: launch_ring_v<LAT, 64, 13, 2, false>(S, Sn, F, rho_next, g, rx, st); break;
    case 2: launch_ring_v<LAT, 64, 8, 3, true>(S, Sn, F, rho_next, g, rx, st); break;
    default: launch_ring_v<LAT, 64, 8, 3, false>(S, Sn, F, rho_next, g, rx, st); break;
    }
}

// Launch variants of the fused kernel (tile height, waves per SIMD the register
// allocation must allow).  The tuner times them on the actual grid.
struct FusedVariant { int ty, occ, pipe; };
constexpr FusedVariant kFusedVariants[] = { {8, 2, 0}, {4, 3, 0}, {6, 3, 0}, {4, 2, 1}, {5, 2, 1}, {3, 2, 1}, {4, 4, 0} };
constexpr int kNumFusedVariants = 7;

template <int LAT, int SCH, int TY, int OCC, bool PIPE>
inline void launch_fused_v(const double* S, double* Sn, const double* rho, const double* mu, double* rho_next,
                           const Grid& g, const Relax& rx, hipStream_t st)
{
    const TileGeom t = fused_tiles(TY, g, LAT == 1);
    const unsigned nb = (unsigned)(t.ntx * t.nty * t.nsz);
    if (rx.omo == 0.0 && !rx.mrt)
        hipLaunchKernelGGL((k_fused<LAT, SCH, TY, OCC, PIPE, true>), dim3(nb), dim3((FX + 2) * (TY + 2)), 0, st, S,
                           Sn, rho, mu, rho_next, g, t, rx);
    else
        hipLaunchKernelGGL((k_fused<LAT, SCH, TY, OCC, PIPE, false>), dim3(nb), dim3((FX + 2) * (TY + 2)), 0, st, S,
                           Sn, rho, mu, rho_next, g, t, rx);
}

template <int LAT, int SCH>
inline void launch_fused_collide(int variant, const double* S, double* Sn, const double* rho, const double* mu,
                                 double* rho_next, const Grid& g, const Relax& rx, hipStream_t st)
{
    switch (variant) {
    case 1: launch_fused_v<LAT, SCH, 4, 3, false>(S, Sn, rho, mu, rho_next, g, rx, st); break;
    case 2: launch_fused_v<LAT, SCH, 6, 3, false>(S, Sn, rho, mu, rho_next, g, rx, st); break;
    case 3: launch_fused_v<LAT, SCH, 4, 2, true>(S, Sn, rho, mu, rho_next, g, rx, st); break;
    case 4: launch_fused_v<LAT, SCH, 5, 2, true>(S, Sn, rho, mu, rho_next, g, rx, st); break;
    case 5: launch_fused_v<LAT, SCH, 3, 2, true>(S, Sn, rho, mu, rho_next, g, rx, st); break;
    case 6: launch_fused_v<LAT, SCH, 4, 4, false>(S, Sn, rho, mu, rho_next, g, rx, st); break;
    default: launch_fused_v<LAT, SCH, 8, 2, false>(S, Sn, rho, mu, rho_next, g, rx, st); break;
    }
}

}  // namespace lbm
