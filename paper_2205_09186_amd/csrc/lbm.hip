// lbm.hip -- C ABI (include/lbm.h) of the gfx950 chemical-potential multiphase
// LBM step (arXiv 2205.09186): context, workspace layout, launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_batch.hpp"
#include "lbm_eos_host.hpp"
#include "lbm_fused.hpp"
#include "lbm_kernels.hpp"
#include "lbm_mlp.hpp"

using namespace lbm;

namespace {

thread_local std::string g_thread_error;

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t S0, S1, rho0, rho1, mu, force, ringsum, zring, grho, gmu, lap, wtmp, wl, wb, partial, result, total;
    long long nparts;
};

PR eos_constants(const lbm_params* p)
{
    PR e;
    e.a = p->a > 0.0 ? p->a : 2.0 / 49.0;
    e.b = p->b > 0.0 ? p->b : 2.0 / 21.0;
    e.R = p->R > 0.0 ? p->R : 1.0;
    e.omega = p->omega > 0.0 ? p->omega : 0.344;
    return e;
}

const char* validate(const lbm_params* p)
{
    if (!p) return "params is NULL";
    if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q19) return "unknown lattice";
    if (p->nx < 4 || p->ny < 4) return "nx and ny must be >= 4";
    if (p->lattice == LBM_D2Q9 && p->nz != 1) return "D2Q9 needs nz == 1";
    if (p->lattice == LBM_D3Q19 && p->nz < 4) return "D3Q19 needs nz >= 4";
    if ((long long)p->nx * p->ny * p->nz > (1LL << 40)) return "grid too large";
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return "tau must be > 0.5";
    if (!(p->Tr > 0.0 && p->Tr < 1.0)) return "Tr must lie in (0, 1)";
    if (!(p->k > 0.0) || !std::isfinite(p->k)) return "k must be > 0";
    if (!(p->kappa > 0.0) || !std::isfinite(p->kappa)) return "kappa must be > 0";
    if (p->scheme < LBM_CD2 || p->scheme > LBM_E10) return "unknown scheme";
    if (p->scheme == LBM_E10 && p->lattice == LBM_D3Q19) return "E10 is defined in two dimensions only";
    if (p->a < 0.0 || p->b < 0.0 || p->R < 0.0 || p->omega < 0.0) return "negative EOS constant";
    if (p->collision != LBM_SRT && p->collision != LBM_MRT) return "unknown collision operator";
    if (p->collision == LBM_MRT && p->lattice != LBM_D2Q9) return "the MRT collision is defined for D2Q9 (Eq 3)";
    for (double s : { p->s_e, p->s_eps, p->s_q })
        if (!(s == 0.0 || (s > 0.0 && s < 2.0))) return "MRT rates must lie in (0, 2) (0 selects the default)";
    if (p->wall != 0 && p->wall != 1) return "wall must be 0 or 1";
    if (p->wall && p->scheme > LBM_CD6) return "walls take the central schemes CD2, CD4, CD6 (Appendix)";
    if (!std::isfinite(p->mu_wall)) return "mu_wall must be finite";
    return nullptr;
}

// Relaxation rates of Eq 1: SRT 1/tau; MRT the diagonal S of Eq 5 with the
// values of Sec 2.1 unless given, divided by the squared row norms of M.
Relax relax_of(const lbm_params* p)
{
    Relax r{};
    r.omo = 1.0 - 1.0 / p->tau;
    r.mrt = p->collision == LBM_MRT ? 1 : 0;
    const double se = p->s_e > 0.0 ? p->s_e : 1.64, seps = p->s_eps > 0.0 ? p->s_eps : 1.54;
    const double sq = p->s_q > 0.0 ? p->s_q : 1.7, snu = 1.0 / p->tau;
    const double S[9] = { 1.0, se, seps, 1.0, sq, 1.0, sq, snu, snu };
    for (int k = 0; k < 9; ++k) r.sd[k] = S[k] / kMrtNorm2[k];
    return r;
}

// Element stride between the Q population arrays: N rounded up to 512 bytes
// plus 4160 elements (32.5 KiB), so that the arrays do not start at the same
// offset modulo large powers of two.  On 256^3 this makes the D3Q19 collide
// kernels about 4% faster than unpadded arrays.
constexpr long long kPopPad = 4160;
long long pop_stride(long long N) { return (N + 63) / 64 * 64 + kPopPad; }

Layout layout_of(const lbm_params* p)
{
    Layout L{};
    const long long N = (long long)p->nx * p->ny * p->nz;
    const int Q = p->lattice == LBM_D2Q9 ? 9 : 19;
    const int dim = p->lattice == LBM_D2Q9 ? 2 : 3;
    const bool compact = is_compact(p->scheme);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.S0 = take(sizeof(double) * Q * pop_stride(N));
    L.S1 = take(sizeof(double) * Q * pop_stride(N));
    L.rho0 = take(sizeof(double) * N);
    L.rho1 = take(sizeof(double) * N);
    L.mu = take(sizeof(double) * N);
    if (N < (1LL << 29)) L.force = take(sizeof(double) * dim * N);
    if (N < (1LL << 29) && p->nx % 64 == 0 && p->ny % kTileTY == 0) {
        Grid g{};
        g.nx = p->nx; g.ny = p->ny; g.nz = p->nz;
        L.ringsum = take(sizeof(double) * ringsum_doubles(g, dim == 3));
        // the z-ring segments of the 3D tile collide (64x16 tiles, no walls)
        if (dim == 3 && !p->wall && p->ny % kZringTY == 0) L.zring = take(sizeof(double) * zring_doubles(g));
    }
    if (p->wall) {
        L.wl = take(N);
        L.wb = take(sizeof(unsigned) * N);
    }
    if (compact) {
        L.grho = take(sizeof(double) * dim * N);
        L.gmu = take(sizeof(double) * dim * N);
        L.lap = take(sizeof(double) * dim * N);    // one term per axis
        L.wtmp = take(sizeof(double) * dim * N);   // one scratch per axis
    }
    L.nparts = (N + 255) / 256;
    L.partial = take(sizeof(double) * 2 * L.nparts);
    L.result = take(sizeof(double) * 2);
    L.total = off;
    return L;
}

}  // namespace

struct lbm_ctx {
    lbm_params p;
    Grid g{};
    Eos eos;
    int Q, dim;
    Relax rx;        // collision of Eq 1 (SRT or D2Q9 MRT)
    hipStream_t stream;
    char* ws;
    Layout L;
    double *S[2], *rhob[2], *mu, *force, *ringsum, *grho, *gmu, *lap, *wtmp, *partial, *result;
    double* zring = nullptr;     // z-ring segment ends of the tile collide (zr variants)
    unsigned* wbits = nullptr;   // wetting boundary: per-node bounce-back mask of the fast path
    int cur;        // index of the buffers holding the current state (S and rho)
    long steps;
    std::string err;
    std::string vname;   // last lbm_variant_name result
    // compact-scheme line geometry per axis
    LineGeom lines[3];
    double z, zscale;
    bool fused;     // fast path: the collide kernel also forms the next density
    int variant = 0;  // launch variant of the fused kernel
    // tile-collide variants this grid and scheme can run (kTileVariants
    // entries; the fused chemical-potential/force march only for the CD
    // schemes in 3D without walls)
    std::vector<TileVariant> tiles;
    // two-step launch graph replayed by lbm_step (captured on a private stream,
    // launched on the context's stream); graph_cur is the state parity it
    // starts from, graph_variant the launch variant it was captured with
    hipGraphExec_t graph = nullptr;
    hipStream_t cap_stream = nullptr;
    int graph_cur = -1, graph_variant = -1;
    bool use_graph = true;
    bool in_batch = false;   // an instance of a batch (stepped by the batched kernel)
    // fewest lines for which the compact line solves take the segmented
    // kernels (lanes across neighbouring lines, coalesced): along y and z
    // where there are enough lines to fill the chip (fewer lines go one
    // wavefront each); along x (rows staged in LDS, RW rows per wavefront)
    // only where rows are many, the whole-row scan being faster on small
    // grids.  LBM_SEG_MIN_LINES sets both (the tests force either path).
    long long seg_min_lines_yz = 4096, seg_min_lines_x = 1LL << 14;
    // y and z lines of up to 1024 points that the segmented kernel does not
    // take: one wavefront per line (LBM_NO_WAVE_LINES: chunked recursions)
    bool wave_lines = true;
    // compact schemes run the per-axis derivative passes concurrently, axis
    // d > 0 on branch stream br[d - 1], forked from and joined to the
    // context's stream by events (LBM_NO_CONC turns it off)
    bool conc = false;
    hipStream_t br[2] = {};
    hipEvent_t bfork = nullptr, bjoin[2] = {};
    // phase timing (lbm_step_timed)
    bool timing = false;
    int nmarks = 0;
    hipEvent_t ev[16] = {};
    const char* phase[16] = {};
};

namespace {

int fail(lbm_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    g_thread_error = msg;
    return code;
}

int hip_check(lbm_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return LBM_OK;
    return fail(c, LBM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Phase boundary for lbm_step_timed: an event on the context's stream.
void mark(lbm_ctx* c, const char* name)
{
    if (!c->timing || c->nmarks >= 16) return;
    (void)hipEventRecord(c->ev[c->nmarks], c->stream);
    c->phase[c->nmarks] = name;
    c->nmarks++;
}

template <int LAT>
void launch_init(lbm_ctx* c, const double* rho0)
{
    hipLaunchKernelGGL(k_init<LAT>, dim3(blocks_for(c->g.N, 256)), dim3(256), 0, c->stream,
                       rho0, c->S[c->cur], c->g);
}

// Compact derivative of field `in` along axis d, delivered to `sink` (stored,
// added, or turned into the force component of Eq 12).
CompactSink sink_of(double* out, int mode, const double* rho = nullptr, const double* grad = nullptr)
{
    CompactSink k{};
    k.out = out; k.mode = mode; k.rho = rho; k.grad = grad;
    return k;
}

void compact_deriv(lbm_ctx* c, const double* in, CompactSink sink, int d)
{
    const LineGeom& lg = c->lines[d];
    const Compact cc = compact_scheme(c->p.scheme);
    // whole lines, one segment of kSegLen points per wave (y, z) or per lane
    // (x, rows staged in LDS), used where there are enough lines to fill the chip
    const bool seg = lg.n <= kSegMaxWavesLong * kSegLen && c->g.N < (1LL << 29) &&
                     (long long)lg.n1 * lg.n2 >= (d == 0 ? c->seg_min_lines_x : c->seg_min_lines_yz);
    if (seg) {
        const int W = (lg.n + kSegLen - 1) / kSegLen;
        const double zS = std::pow(c->z, kSegLen), zLast = std::pow(c->z, lg.n - kSegLen * (W - 1));
        const double zN = std::pow(c->z, lg.n);
        if (d == 0) {
            const XSegGeom q = xseg_geom(lg.n);
            const long long rows = (long long)lg.n1 * lg.n2;
            // up to four wavefronts, within 64 KiB of LDS per workgroup
            const int waves = std::max(1, std::min(4, (int)(65536 / (sizeof(double) * q.RW * q.P))));
            const unsigned blocks = (unsigned)((rows + (long long)waves * q.RW - 1) / ((long long)waves * q.RW));
            hipLaunchKernelGGL(k_compact_xseg, dim3(blocks), dim3(64 * waves), sizeof(double) * waves * q.RW * q.P,
                               c->stream, in, sink, rows, q, cc, c->z, c->zscale, zS, zLast, zN);
        } else {
            const unsigned blocks = (unsigned)(((lg.n1 + 63) / 64) * (long long)lg.n2);
            if (W <= kSegMaxWaves)
                hipLaunchKernelGGL((k_compact_seg<kSegLen, kSegMaxWaves>), dim3(blocks), dim3(64 * W), 0, c->stream,
                                   in, sink, lg, cc, c->z, c->zscale, zS, zLast, zN);
            else
                hipLaunchKernelGGL((k_compact_seg<kSegLen, kSegMaxWavesLong>), dim3(blocks), dim3(64 * W), 0,
                                   c->stream, in, sink, lg, cc, c->z, c->zscale, zS, zLast, zN);
        }
        return;
    }
    if (d > 0 && lg.n <= 64 * kLineSeg && c->wave_lines) {
        // longer lines, or few of them: one wavefront per line, exact (lanes = segments)
        const long long lines = (long long)lg.n1 * lg.n2;
        hipLaunchKernelGGL(k_compact_wave, dim3((unsigned)((lines + 3) / 4)), dim3(256), 0, c->stream, in, sink, lg,
                           cc, c->z, c->zscale);
        return;
    }
    if (d == 0 && lg.n <= 4096 && lg.K <= kScanWarm) {
        // whole rows, one wavefront each, the row and its forward results in
        // LDS (2 nx doubles per wavefront, at most 64 KiB per workgroup)
        const int waves = lg.n <= 1024 ? 4 : 1;
        const long long rows = (long long)lg.n1 * lg.n2;
        hipLaunchKernelGGL(k_compact_x, dim3((unsigned)((rows + waves - 1) / waves)), dim3(64 * waves),
                           sizeof(double) * waves * 2 * lg.n, c->stream, in, sink, lg.n, rows, cc, c->z, c->zscale);
        return;
    }
    const long long items = (long long)lg.n1 * lg.n2 * lg.nch;
    hipLaunchKernelGGL(k_compact_fwd, dim3(blocks_for(items, 256)), dim3(256), 0, c->stream,
                       in, c->wtmp, lg, cc, c->z);
    hipLaunchKernelGGL(k_compact_bwd, dim3(blocks_for(items, 256)), dim3(256), 0, c->stream,
                       c->wtmp, sink, lg, c->z, c->zscale);
}

// Releases the branch streams and events; the axes then run in sequence.
void drop_branches(lbm_ctx* c)
{
    for (int k = 0; k < 2; ++k) {
        if (c->br[k]) (void)hipStreamDestroy(c->br[k]);
        if (c->bjoin[k]) (void)hipEventDestroy(c->bjoin[k]);
        c->br[k] = nullptr;
        c->bjoin[k] = nullptr;
    }
    if (c->bfork) (void)hipEventDestroy(c->bfork);
    c->bfork = nullptr;
    c->conc = false;
}

// fn(d) for every axis d.  With c->conc the axes run concurrently: axis 0
// on the context's stream, axis d > 0 on branch stream br[d - 1] with its own
// scratch; the branches fork from and join the context's stream by events
// (inside a graph capture this makes parallel branches of the graph).
template <class Fn>
void per_axis(lbm_ctx* c, int dim, Fn fn)
{
    if (!c->conc || dim == 1) {
        for (int d = 0; d < dim; ++d) fn(d);
        return;
    }
    hipStream_t main = c->stream;
    double* w0 = c->wtmp;
    (void)hipEventRecord(c->bfork, main);
    for (int k = 0; k < dim - 1; ++k) (void)hipStreamWaitEvent(c->br[k], c->bfork, 0);
    for (int d = 0; d < dim; ++d) {
        c->stream = d == 0 ? main : c->br[d - 1];
        c->wtmp = w0 + d * c->g.N;
        fn(d);
    }
    c->stream = main;
    c->wtmp = w0;
    for (int k = 0; k < dim - 1; ++k) {
        (void)hipEventRecord(c->bjoin[k], c->br[k]);
        (void)hipStreamWaitEvent(main, c->bjoin[k], 0);
    }
}

// Compact schemes: G[rho] into grho, the Laplacian D(D rho) summed over the
// axes, then mu_hat.
void compact_mu(lbm_ctx* c, const double* rho, int dim)
{
    if (c->conc) {
        // each axis: G_d[rho], then its term D_d(G_d[rho]) of the Laplacian;
        // mu_hat then sums the terms in axis order
        const long long N = c->g.N;
        per_axis(c, dim, [&](int d) {
            compact_deriv(c, rho, sink_of(c->grho + d * N, C_STORE), d);
            compact_deriv(c, c->grho + d * N, sink_of(c->lap + d * N, C_STORE), d);
        });
        hipLaunchKernelGGL(k_mu_sum, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream, rho, c->lap, dim, N,
                           c->eos, c->mu);
        return;
    }
    for (int d = 0; d < dim; ++d) compact_deriv(c, rho, sink_of(c->grho + d * c->g.N, C_STORE), d);
    // the last axis's term completes the Laplacian and forms mu_hat (Eq 16)
    for (int d = 0; d < dim - 1; ++d)
        compact_deriv(c, c->grho + d * c->g.N, sink_of(c->lap, d > 0 ? C_ADD : C_STORE), d);
    CompactSink mu_sink = sink_of(c->mu, C_MU, rho, c->lap);
    mu_sink.eos = c->eos;
    compact_deriv(c, c->grho + (dim - 1) * c->g.N, mu_sink, dim - 1);
}

// rho of the current state, then the chemical potential and (compact schemes)
// the gradient fields that the force needs.  On the fast path rho is already
// in rhob[cur] (formed by the last collide) and is left as it is, so that an
// observation does not perturb the state.
template <int LAT, int SCH>
void launch_fields(lbm_ctx* c)
{
    constexpr int DIM = Lat<LAT>::DIM;
    const double* S = c->S[c->cur];
    double* rho = c->rhob[c->cur];
    if (!c->fused)
        hipLaunchKernelGGL(k_rho<LAT>, dim3(blocks_for(c->g.N, 256)), dim3(256), 0, c->stream, S, rho, c->g);
    if (c->g.wl)        // density of the solid layers, Eq A.1, layer after layer
        for (int l = 1; l <= radius(SCH); ++l)
            hipLaunchKernelGGL(k_wall_rho<LAT>, dim3(blocks_for(c->g.N, 256)), dim3(256), 0, c->stream,
                               rho, c->g, l);
    if constexpr (is_compact(SCH)) {
        compact_mu(c, rho, DIM);
        per_axis(c, DIM, [&](int d) { compact_deriv(c, c->mu, sink_of(c->gmu + d * c->g.N, C_STORE), d); });
    } else {
        hipLaunchKernelGGL((k_mu<DIM, SCH>), dim3(blocks_for(c->g.N, 256)), dim3(256), 0, c->stream,
                           rho, c->mu, c->g, c->eos);
    }
}

template <int LAT, int SCH>
void launch_step(lbm_ctx* c)
{
    if (c->fused) {
        // rho of the current state is already in rhob[cur] (written by the
        // previous step's collide or at initialisation); the force pass for
        // the scheme, then the ring collide (or, for the explicit CD schemes,
        // the collide that forms the force itself)
        constexpr int DIM = Lat<LAT>::DIM;
        const double* rho = c->rhob[c->cur];
        constexpr bool CD = SCH == CD2 || SCH == CD4 || SCH == CD6;
        if constexpr (CD) {
            if (c->g.wl) {
                // wetting boundary: the solid layers' density (Eq A.1), the
                // stencil passes, then the tile collide with bounce-back
                mark(c, "k_wall_rho");
                for (int l = 1; l <= radius(SCH); ++l)
                    hipLaunchKernelGGL(k_wall_rho<LAT>, dim3(blocks_for(c->g.N, 256)), dim3(256), 0, c->stream,
                                       c->rhob[c->cur], c->g, l);
                mark(c, "k_mu_march");
                launch_mu_march<DIM, SCH>(rho, c->mu, c->g, c->eos, c->stream);
                mark(c, "k_force_march");
                launch_force_march<DIM, SCH>(rho, c->mu, c->force, c->g, c->eos, c->stream);
                const TileVariant& tv = c->tiles[c->variant];
                mark(c, "k_tile");
                launch_tile<LAT>(tv, c->S[c->cur], c->S[1 - c->cur], c->force, c->rhob[1 - c->cur],
                                 c->ringsum, c->g, c->rx, c->stream, c->wbits);
                mark(c, "k_fix");
                launch_fix<LAT>(tv, c->rhob[1 - c->cur], c->ringsum, c->g, c->stream);
                mark(c, nullptr);
                c->cur = 1 - c->cur;
                return;
            }
        }
        const int rv = CD ? c->variant - kNumFusedVariants : c->variant;
        const TileVariant* tv = rv >= kNumRingVariants ? &c->tiles[rv - kNumRingVariants] : nullptr;
        if constexpr (CD && DIM == 3) {
            if (tv && tv->mf) {
                // chemical potential and force in one march, then the tile collide
                mark(c, "k_mf");
                launch_mf<SCH>(tv->ty, rho, c->force, c->g, c->eos, c->stream);
                mark(c, "k_tile");
                launch_tile<LAT>(*tv, c->S[c->cur], c->S[1 - c->cur], c->force, c->rhob[1 - c->cur], c->ringsum,
                                 c->g, c->rx, c->stream, nullptr, c->zring);
                mark(c, "k_fix");
                launch_fix<LAT>(*tv, c->rhob[1 - c->cur], c->ringsum, c->g, c->stream, c->zring);
                mark(c, nullptr);
                c->cur = 1 - c->cur;
                return;
            }
        }
        if constexpr (!is_compact(SCH)) {
            mark(c, "k_mu_march");
            launch_mu_march<DIM, SCH>(rho, c->mu, c->g, c->eos, c->stream);
        }
        if constexpr (CD) {
            if (c->variant < kNumFusedVariants) {
                mark(c, "k_fused");
                launch_fused_collide<LAT, SCH>(c->variant, c->S[c->cur], c->S[1 - c->cur], rho, c->mu,
                                               c->rhob[1 - c->cur], c->g, c->rx, c->stream);
                mark(c, nullptr);
                c->cur = 1 - c->cur;
                return;
            }
        }
        if constexpr (!is_compact(SCH)) {
            mark(c, "k_force_march");
            launch_force_march<DIM, SCH>(rho, c->mu, c->force, c->g, c->eos, c->stream);
        } else {
            mark(c, "compact derivatives+mu+force");
            compact_mu(c, rho, DIM);
            per_axis(c, DIM, [&](int d) {
                compact_deriv(c, c->mu, sink_of(c->force + d * c->g.N, C_FORCE, rho, c->grho + d * c->g.N), d);
            });
        }
        if (tv) {
            mark(c, "k_tile");
            launch_tile<LAT>(*tv, c->S[c->cur], c->S[1 - c->cur], c->force, c->rhob[1 - c->cur], c->ringsum, c->g,
                             c->rx, c->stream, nullptr, c->zring);
            mark(c, "k_fix");
            launch_fix<LAT>(*tv, c->rhob[1 - c->cur], c->ringsum, c->g, c->stream, c->zring);
        } else {
            mark(c, "k_ring");
            launch_ring_collide<LAT>(rv, c->S[c->cur], c->S[1 - c->cur], c->force, c->rhob[1 - c->cur], c->g, c->rx,
                                     c->stream);
        }
        mark(c, nullptr);
        c->cur = 1 - c->cur;
        return;
    }
    mark(c, is_compact(SCH) ? "rho+compact derivatives+mu" : "k_rho+k_mu");
    launch_fields<LAT, SCH>(c);
    mark(c, "k_collide");
    hipLaunchKernelGGL((k_collide<LAT, SCH>), dim3(blocks_for(c->g.N, 256)), dim3(256), 0, c->stream,
                       c->S[c->cur], c->S[1 - c->cur], c->rhob[c->cur], c->mu, c->grho, c->gmu, c->g,
                       c->rx);
    mark(c, nullptr);
    c->cur = 1 - c->cur;
}

template <int LAT, int SCH>
void launch_macros(lbm_ctx* c, double* orho, double* ovx, double* ovy, double* ovz)
{
    launch_fields<LAT, SCH>(c);
    hipLaunchKernelGGL((k_macros<LAT, SCH>), dim3((unsigned)c->L.nparts), dim3(256), 0, c->stream,
                       c->S[c->cur], c->rhob[c->cur], c->mu, c->grho, c->gmu, c->g, orho, ovx, ovy, ovz,
                       c->partial);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, c->stream, c->partial, c->L.nparts, c->result);
}

// Runtime (lattice, scheme) -> template dispatch.
template <template <int, int> class Op, typename... A>
void dispatch(int lat, int sch, A... a)
{
#define LBM_CASE(L_, S_) case S_: Op<L_, S_>::run(a...); return;
    if (lat == LBM_D2Q9) {
        switch (sch) {
            LBM_CASE(0, 0) LBM_CASE(0, 1) LBM_CASE(0, 2) LBM_CASE(0, 3) LBM_CASE(0, 4)
            LBM_CASE(0, 5) LBM_CASE(0, 6) LBM_CASE(0, 7) LBM_CASE(0, 8) LBM_CASE(0, 9) LBM_CASE(0, 10)
        }
    } else {
        switch (sch) {
            LBM_CASE(1, 0) LBM_CASE(1, 1) LBM_CASE(1, 2) LBM_CASE(1, 3) LBM_CASE(1, 4)
            LBM_CASE(1, 5) LBM_CASE(1, 6) LBM_CASE(1, 7) LBM_CASE(1, 8) LBM_CASE(1, 9)
        }
    }
#undef LBM_CASE
}

template <int LAT, int SCH> struct StepOp { static void run(lbm_ctx* c) { launch_step<LAT, SCH>(c); } };
// mu_hat (and compact gradient fields) of the current state, then the force.
template <int LAT, int SCH>
void launch_force(lbm_ctx* c, double* F)
{
    launch_fields<LAT, SCH>(c);
    hipLaunchKernelGGL((k_force_node<LAT, SCH>), dim3(blocks_for(c->g.N, 256)), dim3(256), 0, c->stream,
                       c->rhob[c->cur], c->mu, c->grho, c->gmu, c->g, F);
}

template <int LAT, int SCH>
void launch_gradient(lbm_ctx* c, const double* in, double* grad, double* lap)
{
    constexpr int DIM = Lat<LAT>::DIM;
    if constexpr (is_compact(SCH)) {
        for (int d = 0; d < DIM; ++d) compact_deriv(c, in, sink_of(grad + d * c->g.N, C_STORE), d);
        if (lap)
            for (int d = 0; d < DIM; ++d)
                compact_deriv(c, grad + d * c->g.N, sink_of(lap, d > 0 ? C_ADD : C_STORE), d);
    } else {
        hipLaunchKernelGGL((k_gradlap<DIM, SCH>), dim3(blocks_for(c->g.N, 256)), dim3(256), 0, c->stream,
                           in, grad, lap, c->g);
    }
}

template <int LAT, int SCH> struct ForceOp { static void run(lbm_ctx* c, double* F) { launch_force<LAT, SCH>(c, F); } };
template <int LAT, int SCH> struct GradOp {
    static void run(lbm_ctx* c, const double* in, double* g, double* l) { launch_gradient<LAT, SCH>(c, in, g, l); }
};

template <int LAT, int SCH> struct MacrosOp {
    static void run(lbm_ctx* c, double* r, double* x, double* y, double* z) { launch_macros<LAT, SCH>(c, r, x, y, z); }
};

void set_lines(lbm_ctx* c)
{
    const int n[3] = { c->p.nx, c->p.ny, c->p.nz };
    const long long st[3] = { 1, (long long)c->p.nx, (long long)c->p.nx * c->p.ny };
    for (int d = 0; d < 3; ++d) {
        LineGeom& lg = c->lines[d];
        const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
        lg.n = n[d]; lg.sa = st[d];
        lg.n1 = n[o1]; lg.s1 = st[o1];
        lg.n2 = n[o2]; lg.s2 = st[o2];
        // chunk length: long chunks waste less on the K-point warm-up, short
        // ones give more threads; aim at ~2^18 threads per axis, C in [16, 128]
        const long long pts = (long long)lg.n * lg.n1 * lg.n2;
        lg.C = (int)std::max(16LL, std::min(128LL, pts >> 18));
        lg.nch = (lg.n + lg.C - 1) / lg.C;
        lg.K = 0;
    }
    if (is_compact(c->p.scheme)) {
        const Compact cc = compact_scheme(c->p.scheme);
        c->z = (-1.0 + std::sqrt(1.0 - 4.0 * cc.al * cc.al)) / (2.0 * cc.al);
        c->zscale = 1.0 + c->z * c->z;
        const int K = (int)std::ceil(std::log(1e-18) / std::log(std::fabs(c->z)));
        for (int d = 0; d < 3; ++d) c->lines[d].K = K;
    } else {
        c->z = 0.0; c->zscale = 1.0;
    }
}

}  // namespace

// Static scratch of lbm_sum_static: 2 doubles per 256-value workgroup plus the
// two results, for at most kStaticSumMaxN values (4 MiB per device, held until
// the process ends).  Host code never uses this name as an address: each
// device's copy is reached through the pointer static_sum_scratch() takes from
// hipGetSymbolAddress with that device current.
constexpr long long kStaticSumMaxN = 1LL << 26;
constexpr long long kStaticSumDoubles = 2 * (kStaticSumMaxN / 256) + 2;
static __device__ __align__(256) double scratch[kStaticSumDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device of stream st (the current device
// for the null stream), looked up once per device with that device current.
int static_sum_scratch(hipStream_t st, double** out)
{
    int cur = 0, dev = 0;
    int r = hip_check(nullptr, hipGetDevice(&cur), "hipGetDevice");
    if (r) return r;
    dev = cur;
    if (st) {
        r = hip_check(nullptr, hipStreamGetDevice(st, &dev), "hipStreamGetDevice");
        if (r) return r;
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, LBM_EINVAL, "lbm_sum_static: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        if (dev != cur) {
            r = hip_check(nullptr, hipSetDevice(dev), "hipSetDevice");
            if (r) return r;
        }
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) (void)hipSetDevice(cur);
        r = hip_check(nullptr, e, "hipGetSymbolAddress(scratch)");
        if (r) return r;
        if (!p) return fail(nullptr, LBM_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_params* p)
{
    if (validate(p)) return 0;
    return layout_of(p).total;
}

}  // extern "C"

namespace {

// Shared by lbm_init and lbm_init_wall; solid is nullptr without walls and
// lies where rho0 lies (host or device).
int init_ctx(const lbm_params* p, const double* rho0, const unsigned char* solid, int rho0_on_device,
             void* d_workspace, size_t ws_bytes, void* hip_stream, lbm_ctx** out)
{
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char* why = validate(p)) return fail(nullptr, LBM_EINVAL, why);
    if (!rho0) return fail(nullptr, LBM_EINVAL, "rho0 is NULL");
    if (!d_workspace) return fail(nullptr, LBM_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
        return fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
    const Layout L = layout_of(p);
    if (ws_bytes < L.total)
        return fail(nullptr, LBM_ENOSPC, "workspace too small: need " + std::to_string(L.total) + " bytes");

    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_EHIP, "out of host memory");
    c->p = *p;
    c->Q = p->lattice == LBM_D2Q9 ? 9 : 19;
    c->dim = p->lattice == LBM_D2Q9 ? 2 : 3;
    c->g.nx = p->nx; c->g.ny = p->ny; c->g.nz = p->nz;
    c->g.nxy = (long long)p->nx * p->ny;
    c->g.N = c->g.nxy * p->nz;
    c->g.ps = pop_stride(c->g.N);
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->ws = static_cast<char*>(d_workspace);
    c->L = L;
    c->S[0] = reinterpret_cast<double*>(c->ws + L.S0);
    c->S[1] = reinterpret_cast<double*>(c->ws + L.S1);
    c->rhob[0] = reinterpret_cast<double*>(c->ws + L.rho0);
    c->rhob[1] = reinterpret_cast<double*>(c->ws + L.rho1);
    c->mu = reinterpret_cast<double*>(c->ws + L.mu);
    c->force = c->g.N < (1LL << 29) ? reinterpret_cast<double*>(c->ws + L.force) : nullptr;
    c->ringsum = (c->force && tile_fits(c->g, kTileTY)) ? reinterpret_cast<double*>(c->ws + L.ringsum) : nullptr;
    c->zring = (c->ringsum && c->dim == 3 && !p->wall && p->ny % kZringTY == 0)
                   ? reinterpret_cast<double*>(c->ws + L.zring) : nullptr;
    const bool compact = is_compact(p->scheme);
    c->grho = compact ? reinterpret_cast<double*>(c->ws + L.grho) : nullptr;
    c->gmu = compact ? reinterpret_cast<double*>(c->ws + L.gmu) : nullptr;
    c->lap = compact ? reinterpret_cast<double*>(c->ws + L.lap) : nullptr;
    c->wtmp = compact ? reinterpret_cast<double*>(c->ws + L.wtmp) : nullptr;
    unsigned char* wl = p->wall ? reinterpret_cast<unsigned char*>(c->ws + L.wl) : nullptr;
    c->partial = reinterpret_cast<double*>(c->ws + L.partial);
    c->result = reinterpret_cast<double*>(c->ws + L.result);
    c->cur = 0;
    c->steps = 0;
    c->rx = relax_of(p);
    // walls run on the tile collide (central schemes, grids tiled by 64 x 8),
    // else on the node-parallel path
    c->fused = c->g.N < (1LL << 29) && std::getenv("LBM_NO_FUSED") == nullptr &&
               (!p->wall || (p->scheme <= LBM_CD6 && c->ringsum));
    // untuned default for the CD schemes: the ring collide with its own force
    // pass in 3D, the collide that forms the force itself in 2D (fastest of
    // each on 256^3 and 1024^2); the other schemes have only ring variants
    c->variant = (p->lattice == LBM_D3Q19 && p->scheme <= LBM_CD6 && !p->wall) ? kNumFusedVariants : 0;
    if (c->ringsum) {
        const bool mf_ok = p->lattice == LBM_D3Q19 && p->scheme <= LBM_CD6 && !p->wall;
        for (const TileVariant& v : kTileVariants) {
            if (!tile_fits(c->g, v.ty)) continue;
            if (p->lattice == LBM_D2Q9 && v.fz != kTileVariants[0].fz) continue;   // one segment in 2D
            if (v.mf && !mf_ok) continue;
            if (v.zr && !c->zring) continue;
            c->tiles.push_back(v);
        }
    }
    c->use_graph = std::getenv("LBM_NO_GRAPH") == nullptr;
    if (const char* e = std::getenv("LBM_SEG_MIN_LINES")) c->seg_min_lines_yz = c->seg_min_lines_x = std::atoll(e);
    c->wave_lines = std::getenv("LBM_NO_WAVE_LINES") == nullptr;
    // measured faster at every size from 100^2 to 256^3 (2D 1024^2 by 15%)
    c->conc = compact && std::getenv("LBM_NO_CONC") == nullptr;
    set_lines(c);
    if (c->conc) {
        int r = LBM_OK;
        for (int k = 0; k < c->dim - 1 && r == LBM_OK; ++k) {
            r = hip_check(c, hipStreamCreateWithFlags(&c->br[k], hipStreamNonBlocking), "branch stream");
            if (r == LBM_OK)
                r = hip_check(c, hipEventCreateWithFlags(&c->bjoin[k], hipEventDisableTiming), "branch event");
        }
        if (r == LBM_OK) r = hip_check(c, hipEventCreateWithFlags(&c->bfork, hipEventDisableTiming), "fork event");
        if (r != LBM_OK) { lbm_free(c); return r; }
    }

    // equation of state in mesh units (Eq 16): k^2 psi'
    const PR e = eos_constants(p);
    double Tc, rc, pc;
    pr_critical(e, Tc, rc, pc);
    const double T = p->Tr * Tc;
    const double aa = e.a * pr_alpha(p->Tr, e.omega);
    const double k2 = p->k * p->k;
    c->eos.k2RT = k2 * e.R * T;
    c->eos.k2c = k2 * aa / (2.0 * std::sqrt(2.0) * e.b);
    c->eos.k2aa = k2 * aa;
    c->eos.b = e.b;
    c->eos.kappa = p->kappa;
    c->eos.mu_wall = p->mu_wall;

    // initial density: validate on the host, stage through the rho buffer
    const long long N = c->g.N;
    const double rho_max = 1.0 / e.b;
    int rc_ = LBM_OK;
    if (wl) {
        // the solid mask into the layer map: 0 fluid, kDeepSolid solid, then
        // the layers 1..r counted from the fluid
        rc_ = hip_check(c, hipMemcpyAsync(wl, solid, N, rho0_on_device ? hipMemcpyDeviceToDevice
                                                                        : hipMemcpyHostToDevice, c->stream),
                        "copy solid mask");
        if (rc_ == LBM_OK) {
            hipLaunchKernelGGL(k_wall_mark, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream, wl, N);
            for (int l = 1; l <= radius(p->scheme); ++l) {
                if (p->lattice == LBM_D2Q9)
                    hipLaunchKernelGGL(k_wall_layer<0>, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream, wl, c->g, l);
                else
                    hipLaunchKernelGGL(k_wall_layer<1>, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream, wl, c->g, l);
            }
            c->g.wl = wl;
            c->wbits = reinterpret_cast<unsigned*>(c->ws + L.wb);
            if (p->lattice == LBM_D2Q9)
                hipLaunchKernelGGL(k_wall_bits<0>, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream, wl, c->wbits, c->g);
            else
                hipLaunchKernelGGL(k_wall_bits<1>, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream, wl, c->wbits, c->g);
        }
    }
    if (rc_ == LBM_OK && !rho0_on_device) {
        for (long long n = 0; n < N; ++n) {
            if (solid && solid[n]) continue;       // no density is read on solid nodes
            const double r = rho0[n];
            if (!(r > 0.0 && r < rho_max)) { rc_ = fail(c, LBM_EINVAL, "rho0 must be finite and in (0, 1/b)"); break; }
        }
        if (rc_ == LBM_OK)
            rc_ = hip_check(c, hipMemcpyAsync(c->rhob[1], rho0, sizeof(double) * N, hipMemcpyHostToDevice,
                                              c->stream), "copy rho0");
    } else if (rc_ == LBM_OK) {
        rc_ = hip_check(c, hipMemcpyAsync(c->rhob[1], rho0, sizeof(double) * N, hipMemcpyDeviceToDevice,
                                          c->stream), "copy rho0");
        // the same range check on the device: nodes outside (0, 1/b), counted
        if (rc_ == LBM_OK) {
            hipLaunchKernelGGL(k_check_rho, dim3((unsigned)L.nparts), dim3(256), 0, c->stream, c->rhob[1], wl, N,
                               rho_max, c->partial);
            hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, c->stream, c->partial, L.nparts, c->result);
            double h[2] = { 0.0, 0.0 };
            rc_ = hip_check(c, hipMemcpyAsync(h, c->result, sizeof(h), hipMemcpyDeviceToHost, c->stream),
                            "rho0 check copy");
            if (rc_ == LBM_OK) rc_ = hip_check(c, hipStreamSynchronize(c->stream), "rho0 check sync");
            if (rc_ == LBM_OK && h[1] != 0.0)
                rc_ = fail(c, LBM_EINVAL, "rho0 on device: " + std::to_string((long long)h[1]) +
                                              " node(s) not finite or outside (0, 1/b)");
        }
    }
    if (rc_ == LBM_OK) {
        // populations from rho0, then rho of that state (what the step reads)
        if (p->lattice == LBM_D2Q9) {
            launch_init<0>(c, c->rhob[1]);
            hipLaunchKernelGGL(k_rho<0>, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream, c->S[0], c->rhob[0], c->g);
        } else {
            launch_init<1>(c, c->rhob[1]);
            hipLaunchKernelGGL(k_rho<1>, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream, c->S[0], c->rhob[0], c->g);
        }
        // the step recomputes rho on the node-parallel path; only the fused
        // path (never with walls) reads this one
        rc_ = hip_check(c, hipGetLastError(), "init launch");
    }
    if (rc_ == LBM_OK) rc_ = hip_check(c, hipStreamSynchronize(c->stream), "init sync");
    if (rc_ != LBM_OK) { lbm_free(c); return rc_; }
    *out = c;
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_init(const lbm_params* p, const double* rho0, int rho0_on_device, void* d_workspace,
             size_t ws_bytes, void* hip_stream, lbm_ctx** out)
{
    if (p && p->wall) {
        if (out) *out = nullptr;
        return fail(nullptr, LBM_EINVAL, "wall = 1 needs lbm_init_wall and a solid mask");
    }
    return init_ctx(p, rho0, nullptr, rho0_on_device, d_workspace, ws_bytes, hip_stream, out);
}

int lbm_init_wall(const lbm_params* p, const double* rho0, const unsigned char* solid, int on_device,
                  void* d_workspace, size_t ws_bytes, void* hip_stream, lbm_ctx** out)
{
    if (!p || !p->wall) {
        if (out) *out = nullptr;
        return fail(nullptr, LBM_EINVAL, "lbm_init_wall needs wall = 1");
    }
    if (!solid) {
        if (out) *out = nullptr;
        return fail(nullptr, LBM_EINVAL, "solid is NULL");
    }
    return init_ctx(p, rho0, solid, on_device, d_workspace, ws_bytes, hip_stream, out);
}

namespace {

// Capture the launch sequence of two consecutive steps (state parity cur, then
// 1 - cur) into an executable graph.
int capture_pair(lbm_ctx* c)
{
    if (c->graph) { (void)hipGraphExecDestroy(c->graph); c->graph = nullptr; }
    int r;
    if (!c->cap_stream &&
        (r = hip_check(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream")))
        return r;
    hipStream_t user = c->stream;
    const int cur0 = c->cur;
    c->stream = c->cap_stream;
    hipGraph_t g = nullptr;
    r = hip_check(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    if (r == LBM_OK) {
        dispatch<StepOp>(c->p.lattice, c->p.scheme, c);
        dispatch<StepOp>(c->p.lattice, c->p.scheme, c);
        r = hip_check(c, hipStreamEndCapture(c->cap_stream, &g), "end capture");
    }
    c->stream = user;
    c->cur = cur0;   // capture only recorded the launches
    if (r == LBM_OK) r = hip_check(c, hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0), "instantiate graph");
    if (g) (void)hipGraphDestroy(g);
    if (r == LBM_OK) { c->graph_cur = cur0; c->graph_variant = c->variant; }
    else c->graph = nullptr;
    return r;
}

}  // namespace

int lbm_step(lbm_ctx* c, long nsteps)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(c, LBM_EINVAL, "nsteps must be >= 0");
    long s = 0;
    if (c->use_graph && nsteps >= 4) {
        if (c->cur != c->graph_cur && c->graph && c->graph_variant == c->variant) {
            // align the parity with the captured pair by one plain step
            dispatch<StepOp>(c->p.lattice, c->p.scheme, c);
            c->steps++;
            s++;
        }
        if (!c->graph || c->graph_variant != c->variant || c->cur != c->graph_cur) {
            if (capture_pair(c) != LBM_OK) {
                // no graph on this runtime: plain launches from here on
                c->use_graph = false;
                (void)hipGetLastError();
            }
        }
        for (; c->use_graph && s + 2 <= nsteps; s += 2) {
            int r = hip_check(c, hipGraphLaunch(c->graph, c->stream), "graph launch");
            if (r) return r;
            c->steps += 2;
        }
    }
    for (; s < nsteps; ++s) {
        dispatch<StepOp>(c->p.lattice, c->p.scheme, c);
        c->steps++;
    }
    return hip_check(c, hipGetLastError(), "step launch");
}

int lbm_macros(lbm_ctx* c, double* rho, double* vx, double* vy, double* vz, int out_on_device)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (c->dim == 2) vz = nullptr;
    const long long N = c->g.N;
    if (out_on_device) {
        dispatch<MacrosOp>(c->p.lattice, c->p.scheme, c, rho, vx, vy, vz);
        int r = hip_check(c, hipGetLastError(), "macros launch");
        if (r) return r;
        return hip_check(c, hipStreamSynchronize(c->stream), "macros sync");
    }
    // host outputs: compute into device scratch (the gradient buffers are free
    // between steps only for compact schemes, so use the two population-sized
    // halves of the idle buffer), then copy
    double* idle = c->S[1 - c->cur];
    double* d_r = idle;
    double* d_x = idle + N;
    double* d_y = idle + 2 * N;
    double* d_z = c->dim == 3 ? idle + 3 * N : nullptr;
    dispatch<MacrosOp>(c->p.lattice, c->p.scheme, c, d_r, d_x, d_y, d_z);
    int r = hip_check(c, hipGetLastError(), "macros launch");
    if (r) return r;
    const size_t b = sizeof(double) * N;
    if (rho && (r = hip_check(c, hipMemcpyAsync(rho, d_r, b, hipMemcpyDeviceToHost, c->stream), "copy rho"))) return r;
    if (vx && (r = hip_check(c, hipMemcpyAsync(vx, d_x, b, hipMemcpyDeviceToHost, c->stream), "copy vx"))) return r;
    if (vy && (r = hip_check(c, hipMemcpyAsync(vy, d_y, b, hipMemcpyDeviceToHost, c->stream), "copy vy"))) return r;
    if (vz && d_z && (r = hip_check(c, hipMemcpyAsync(vz, d_z, b, hipMemcpyDeviceToHost, c->stream), "copy vz")))
        return r;
    return hip_check(c, hipStreamSynchronize(c->stream), "macros sync");
}

int lbm_force(lbm_ctx* c, double* F, double* mu, int out_on_device)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    const long long N = c->g.N;
    // F is formed in the idle population buffer (dim N <= Q N), mu in c->mu
    double* d_F = c->S[1 - c->cur];
    dispatch<ForceOp>(c->p.lattice, c->p.scheme, c, d_F);
    int r = hip_check(c, hipGetLastError(), "force launch");
    if (r) return r;
    const hipMemcpyKind k = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (F && (r = hip_check(c, hipMemcpyAsync(F, d_F, sizeof(double) * c->dim * N, k, c->stream), "copy F")))
        return r;
    if (mu && (r = hip_check(c, hipMemcpyAsync(mu, c->mu, sizeof(double) * N, k, c->stream), "copy mu"))) return r;
    return hip_check(c, hipStreamSynchronize(c->stream), "force sync");
}

int lbm_gradient(lbm_ctx* c, const double* d_in, double* d_grad, double* d_lap)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (!d_in || !d_grad) return fail(c, LBM_EINVAL, "d_in and d_grad must be device arrays");
    if (d_in == d_grad || d_in == d_lap) return fail(c, LBM_EINVAL, "d_in must not alias the outputs");
    dispatch<GradOp>(c->p.lattice, c->p.scheme, c, d_in, d_grad, d_lap);
    return hip_check(c, hipGetLastError(), "gradient launch");
}

int lbm_spurious_max(lbm_ctx* c, double* umax, double* mass)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    dispatch<MacrosOp>(c->p.lattice, c->p.scheme, c, (double*)nullptr, (double*)nullptr, (double*)nullptr,
                       (double*)nullptr);
    int r = hip_check(c, hipGetLastError(), "observables launch");
    if (r) return r;
    double h[2];
    r = hip_check(c, hipMemcpyAsync(h, c->result, sizeof(h), hipMemcpyDeviceToHost, c->stream), "copy result");
    if (r) return r;
    r = hip_check(c, hipStreamSynchronize(c->stream), "observables sync");
    if (r) return r;
    if (umax) *umax = h[0];
    if (mass) *mass = h[1];
    if (!std::isfinite(h[0]) || !std::isfinite(h[1]) || h[0] > std::sqrt(1.0 / 3.0))
        return fail(c, LBM_ENONFINITE, "non-finite state or |v| above the lattice sound speed");
    return LBM_OK;
}

int lbm_populations(lbm_ctx* c, double* f, int out_on_device)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (!f) return fail(c, LBM_EINVAL, "f is NULL");
    // The stored buffer holds post-collision values at their source nodes;
    // the post-streaming state is their pull, staged in the idle buffer.
    const long long N = c->g.N;
    const double* S = c->S[c->cur];
    double* tmp = c->S[1 - c->cur];
    if (c->p.lattice == LBM_D2Q9)
        hipLaunchKernelGGL(k_pull_all<0>, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream, S, tmp, c->g);
    else
        hipLaunchKernelGGL(k_pull_all<1>, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream, S, tmp, c->g);
    int r = hip_check(c, hipGetLastError(), "pull launch");
    if (r) return r;
    r = hip_check(c, hipMemcpyAsync(f, tmp, sizeof(double) * c->Q * N,
                                    out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream),
                  "copy populations");
    if (r) return r;
    return hip_check(c, hipStreamSynchronize(c->stream), "populations sync");
}

long lbm_steps_done(const lbm_ctx* c) { return c ? c->steps : -1; }

namespace {

// Header of a state image: magic, layout version, lattice, nx, ny, nz,
// completed steps, one spare word.
constexpr long long kStateMagic = 0x4554415453424C4CLL;   // "LLBSTATE" read as little-endian bytes
constexpr long long kStateVersion = 1;
constexpr size_t kStateHeader = 64;

}  // namespace

size_t lbm_state_bytes(const lbm_ctx* c)
{
    if (!c) return 0;
    return kStateHeader + sizeof(double) * ((size_t)c->Q + 1) * (size_t)c->g.N;
}

int lbm_save_state(lbm_ctx* c, void* out, int on_device)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (!out) return fail(c, LBM_EINVAL, "out is NULL");
    const long long hdr[8] = { kStateMagic, kStateVersion, c->p.lattice, c->p.nx, c->p.ny, c->p.nz, c->steps, 0 };
    char* o = static_cast<char*>(out);
    const size_t N = (size_t)c->g.N;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    int r = LBM_OK;
    if (on_device)
        r = hip_check(c, hipMemcpyAsync(o, hdr, sizeof hdr, hipMemcpyHostToDevice, c->stream), "state header");
    else
        std::memcpy(o, hdr, sizeof hdr);
    // the Q population arrays (stored with the padded stride) packed one after another
    if (r == LBM_OK)
        r = hip_check(c, hipMemcpy2DAsync(o + kStateHeader, N * sizeof(double), c->S[c->cur],
                                          (size_t)c->g.ps * sizeof(double), N * sizeof(double), (size_t)c->Q, kind,
                                          c->stream), "state populations");
    if (r == LBM_OK)
        r = hip_check(c, hipMemcpyAsync(o + kStateHeader + sizeof(double) * c->Q * N, c->rhob[c->cur],
                                        sizeof(double) * N, kind, c->stream), "state density");
    // always drained before returning: the header copy reads this frame
    const hipError_t se = hipStreamSynchronize(c->stream);
    if (r == LBM_OK) r = hip_check(c, se, "state sync");
    return r;
}

int lbm_load_state(lbm_ctx* c, const void* in, int on_device)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (!in) return fail(c, LBM_EINVAL, "in is NULL");
    if (c->in_batch) return fail(c, LBM_ESTATE, "a batch instance's state belongs to the batch");
    const char* i = static_cast<const char*>(in);
    long long hdr[8];
    if (on_device) {
        int r = hip_check(c, hipMemcpyAsync(hdr, i, sizeof hdr, hipMemcpyDeviceToHost, c->stream), "state header");
        const hipError_t se = hipStreamSynchronize(c->stream);
        if (r == LBM_OK) r = hip_check(c, se, "state header sync");
        if (r) return r;
    } else {
        std::memcpy(hdr, i, sizeof hdr);
    }
    if (hdr[0] != kStateMagic || hdr[1] != kStateVersion) return fail(c, LBM_EINVAL, "not a state image");
    if (hdr[2] != c->p.lattice || hdr[3] != c->p.nx || hdr[4] != c->p.ny || hdr[5] != c->p.nz)
        return fail(c, LBM_EINVAL, "state image of another lattice or grid size");
    if (hdr[6] < 0) return fail(c, LBM_EINVAL, "state image with a negative step count");
    const size_t N = (size_t)c->g.N;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    int r = hip_check(c, hipMemcpy2DAsync(c->S[c->cur], (size_t)c->g.ps * sizeof(double), i + kStateHeader,
                                          N * sizeof(double), N * sizeof(double), (size_t)c->Q, kind, c->stream),
                      "state populations");
    if (r == LBM_OK)
        r = hip_check(c, hipMemcpyAsync(c->rhob[c->cur], i + kStateHeader + sizeof(double) * c->Q * N,
                                        sizeof(double) * N, kind, c->stream), "state density");
    // always drained before returning, so the caller may release the image
    const hipError_t se = hipStreamSynchronize(c->stream);
    if (r == LBM_OK) r = hip_check(c, se, "state sync");
    if (r == LBM_OK) c->steps = (long)hdr[6];
    return r;
}

int lbm_step_timed(lbm_ctx* c, long nsteps, double* ms, int cap, int* nphases)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (nsteps < 1 || !ms || cap < 1 || !nphases) return fail(c, LBM_EINVAL, "bad timing arguments");
    for (int k = 0; k < 16; ++k)
        if (!c->ev[k]) {
            int r = hip_check(c, hipEventCreate(&c->ev[k]), "event create");
            if (r) return r;
        }
    for (int k = 0; k < cap; ++k) ms[k] = 0.0;
    int np = 0;
    c->timing = true;
    for (long s = 0; s < nsteps; ++s) {
        c->nmarks = 0;
        dispatch<StepOp>(c->p.lattice, c->p.scheme, c);
        c->steps++;
        int r = hip_check(c, hipEventSynchronize(c->ev[c->nmarks - 1]), "timing sync");
        if (r) { c->timing = false; return r; }
        np = c->nmarks - 1;
        for (int k = 0; k < np && k < cap; ++k) {
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, c->ev[k], c->ev[k + 1]);
            ms[k] += t / (double)nsteps;
        }
    }
    c->timing = false;
    *nphases = np;
    return hip_check(c, hipGetLastError(), "timed step");
}

int lbm_num_variants(const lbm_ctx* c)
{
    if (!c || !c->fused) return 1;
    if (c->g.wl) return (int)c->tiles.size();   // walls: the tile collide only
    const int tiles = (int)c->tiles.size();
    return (c->p.scheme <= LBM_CD6 ? kNumFusedVariants : 0) + kNumRingVariants + tiles;
}

int lbm_set_variant(lbm_ctx* c, int v)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (v < 0 || v >= lbm_num_variants(c)) return fail(c, LBM_EINVAL, "variant out of range");
    c->variant = v;
    return LBM_OK;
}

const char* lbm_phase_name(const lbm_ctx* c, int k)
{
    if (!c || k < 0 || k >= 15 || !c->phase[k]) return "";
    return c->phase[k];
}

const char* lbm_variant_name(lbm_ctx* c, int v)
{
    if (!c || v < 0 || v >= lbm_num_variants(c)) return "";
    char buf[96];
    int t = v;
    if (!c->g.wl) {
        const bool cd = c->p.scheme <= LBM_CD6;
        if (cd) {
            if (t < kNumFusedVariants) {
                const FusedVariant& f = kFusedVariants[t];
                std::snprintf(buf, sizeof buf, "fused 64x%d occ%d%s", f.ty, f.occ, f.pipe ? " pipe" : "");
                return (c->vname = buf).c_str();
            }
            t -= kNumFusedVariants;
        }
        if (t < kNumRingVariants) {
            const RingVariant& r = kRingVariants[t];
            std::snprintf(buf, sizeof buf, "ring %dx%d occ%d%s", r.tx, r.ty, r.occ, r.pf ? " prefetch" : "");
            return (c->vname = buf).c_str();
        }
        t -= kNumRingVariants;
    }
    const TileVariant& tv = c->tiles[t];
    if (c->dim == 3)
        std::snprintf(buf, sizeof buf, "tile 64x%d z%d%s%s", tv.ty, tv.fz, tv.mf ? " mf" : "", tv.zr ? " zr" : "");
    else std::snprintf(buf, sizeof buf, "tile 64x%d", tv.ty);
    return (c->vname = buf).c_str();
}

void lbm_free(lbm_ctx* c)
{
    if (!c) return;
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    drop_branches(c);
    for (int k = 0; k < 16; ++k)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    delete c;
}

const char* lbm_last_error(const lbm_ctx* c)
{
    if (c) return c->err.c_str();
    return g_thread_error.c_str();
}

int lbm_critical(const lbm_params* p, double* Tc, double* rho_c, double* p_c)
{
    if (!p || !Tc || !rho_c || !p_c) return fail(nullptr, LBM_EINVAL, "NULL argument");
    pr_critical(eos_constants(p), *Tc, *rho_c, *p_c);
    return LBM_OK;
}

int lbm_eos(const lbm_params* p, const double* rho, long n, double* p0, double* mu)
{
    if (!p || !rho || n < 0) return fail(nullptr, LBM_EINVAL, "NULL argument");
    if (!(p->Tr > 0.0 && p->Tr < 1.0)) return fail(nullptr, LBM_EINVAL, "Tr must lie in (0, 1)");
    const PR e = eos_constants(p);
    double Tc, rc, pc;
    pr_critical(e, Tc, rc, pc);
    const double T = p->Tr * Tc, aa = e.a * pr_alpha(p->Tr, e.omega);
    for (long i = 0; i < n; ++i) {
        if (!(rho[i] > 0.0 && rho[i] * e.b < 1.0)) return fail(nullptr, LBM_EINVAL, "density outside (0, 1/b)");
        if (p0) p0[i] = pr_pressure(e, aa, T, rho[i]);
        if (mu) mu[i] = pr_mu(e, aa, T, rho[i]);
    }
    return LBM_OK;
}

int lbm_coexistence(const lbm_params* p, double* rho_g, double* rho_l)
{
    if (!p || !rho_g || !rho_l) return fail(nullptr, LBM_EINVAL, "NULL argument");
    if (!pr_coexistence(eos_constants(p), p->Tr, *rho_g, *rho_l))
        return fail(nullptr, LBM_EINVAL, "no coexistence at this Tr");
    return LBM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched sweep
// ---------------------------------------------------------------------------
struct lbm_batch {
    int n = 0;
    std::vector<lbm_ctx*> ctx;
    std::vector<BInst> inst;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    BInst* d_inst = nullptr;
    BState* d_st = nullptr;
    int* d_blk_inst = nullptr;
    double* d_partial = nullptr;
    BLine* d_lines = nullptr;
    // d_flag[0]: set by k_batch if a launch was not cooperative; d_flag[1]:
    // launches that k_batch completed (h_flag: their read-back), against
    // `launches`, the count the host expects
    int* d_flag = nullptr;
    unsigned launches = 0;
    BState* h_st = nullptr;     // pinned host copies read after every chunk
    int* h_flag = nullptr;
    // the work-item tables hold the instances running when they were built
    // (retired ones then cost nothing); rebuilt between chunks once fewer run
    int nblk_total = 0;
    int nlines = 0;
    int has_compact = 0;
    int table_running = 0;
    std::vector<BLine> all_lines;     // the grid lines of every compact-scheme instance
    int block = kBatchDefaultBlock;   // nodes per node-block item = threads per workgroup
    int grid = 0;                     // workgroups of the cooperative launch
    int max_grid_of[kNumBatchBlocks] = {};
    int form = LBM_BATCH_PERSISTENT;  // launch form
    // chunk launches captured as graphs: the cooperative kernel (or the phase
    // kernels) and the two status read-backs, one graph per (form, chunk
    // length, check interval, tolerance, workgroups, block, and for the phase
    // form the loop steps that carry a check); replayed on the batch's stream
    struct Graph {
        int form, todo, check, grid, block;
        double tol;
        std::vector<char> due;
        hipGraphExec_t exec;
        std::string how;    // the launch mode it reports
    };
    std::vector<Graph> graphs;
    hipStream_t cap_stream = nullptr;
    bool use_graph = true;
    std::string mode = "plain cooperative launches";
    std::string err;
};

namespace {

constexpr long kPhaseChunk = 1000;        // steps per launch sequence of the phase form
constexpr size_t kMaxBatchGraphs = 16;   // cached chunk graphs per batch

struct BatchLayout {
    std::vector<size_t> inst_off;
    size_t tables, total;
    int nblk, nlines;
};

bool batch_layout(const lbm_params* ps, int n, BatchLayout& B, const char** why)
{
    size_t off = 0;
    B.inst_off.resize(n);
    B.nblk = 0;
    B.nlines = 0;
    for (int i = 0; i < n; ++i) {
        if (const char* w = validate(&ps[i])) { *why = w; return false; }
        if (ps[i].lattice != LBM_D2Q9) { *why = "the batched sweep runs D2Q9 instances"; return false; }
        if (ps[i].wall) { *why = "the batched sweep runs periodic instances"; return false; }
        B.inst_off[i] = off;
        off = align_up(off + layout_of(&ps[i]).total);
        const long long N = (long long)ps[i].nx * ps[i].ny;
        // node-block tables sized for the smallest block
        B.nblk += (int)((N + kBatchMinBlock - 1) / kBatchMinBlock);
        if (is_compact(ps[i].scheme)) {
            if (std::max(ps[i].nx, ps[i].ny) > 64 * kLineSeg) {
                *why = "compact-scheme instances of the batched sweep take lines of at most 1024 nodes";
                return false;
            }
            B.nlines += ps[i].nx + ps[i].ny;
        }
    }
    B.tables = off;
    off = align_up(off + sizeof(BInst) * n);
    off = align_up(off + sizeof(BState) * n);
    off = align_up(off + sizeof(int) * B.nblk);
    off = align_up(off + sizeof(double) * B.nblk);
    off = align_up(off + sizeof(BLine) * std::max(1, B.nlines));
    off = align_up(off + 2 * sizeof(int));
    B.total = off;
    return true;
}

int bfail(lbm_batch* b, int code, const std::string& msg)
{
    if (b) b->err = msg;
    g_thread_error = msg;
    return code;
}

int batch_block_index(int block)
{
    for (int k = 0; k < kNumBatchBlocks; ++k)
        if (kBatchBlocks[k] == block) return k;
    return -1;
}

const void* batch_kernel(int block)
{
    switch (block) {
    case 256: return reinterpret_cast<const void*>(k_batch<256>);
    case 1024: return reinterpret_cast<const void*>(k_batch<1024>);
    default: return reinterpret_cast<const void*>(k_batch<512>);
    }
}

// Node-block items of every instance for the batch's block size, uploaded
// with the instance table; synchronises.
hipError_t batch_tables(lbm_batch* b)
{
    // node-block items and compact-scheme lines of the instances still
    // running (by the status last read back); a retired instance keeps its
    // entry in the instance table with no items
    std::vector<int> blk_inst;
    int running = 0, compact = 0;
    for (int i = 0; i < b->n; ++i) {
        BInst& I = b->inst[i];
        const bool run = b->h_st[i].status == B_RUNNING;
        I.blk0 = (int)blk_inst.size();
        I.nblk = run ? (int)((I.g.N + b->block - 1) / b->block) : 0;
        for (int k = 0; k < I.nblk; ++k) blk_inst.push_back(i);
        I.part0 = I.blk0;
        running += run;
        compact |= run && is_compact(I.scheme);
    }
    std::vector<BLine> lines;
    for (const BLine& ln : b->all_lines)
        if (b->h_st[ln.inst].status == B_RUNNING) lines.push_back(ln);
    b->nblk_total = (int)blk_inst.size();
    b->nlines = (int)lines.size();
    b->has_compact = compact;
    b->table_running = running;
    hipError_t e = hipMemcpyAsync(b->d_inst, b->inst.data(), sizeof(BInst) * b->n, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !blk_inst.empty())
        e = hipMemcpyAsync(b->d_blk_inst, blk_inst.data(), sizeof(int) * blk_inst.size(), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess && !lines.empty())
        e = hipMemcpyAsync(b->d_lines, lines.data(), sizeof(BLine) * lines.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e;
}

void drop_graphs(lbm_batch* b)
{
    for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
}

// The kernel node of a graph carries the cooperative launch attribute, or
// gets it; anything else is refused (the graph is not used).
hipError_t ensure_cooperative(hipGraph_t g)
{
    size_t num = 0;
    hipError_t e = hipGraphGetNodes(g, nullptr, &num);
    if (e != hipSuccess) return e;
    std::vector<hipGraphNode_t> nodes(num);
    e = hipGraphGetNodes(g, nodes.data(), &num);
    int kernels = 0;
    for (size_t k = 0; k < num && e == hipSuccess; ++k) {
        hipGraphNodeType t;
        e = hipGraphNodeGetType(nodes[k], &t);
        if (e != hipSuccess || t != hipGraphNodeTypeKernel) continue;
        ++kernels;
        hipKernelNodeAttrValue v{};
        e = hipGraphKernelNodeGetAttribute(nodes[k], hipKernelNodeAttributeCooperative, &v);
        if (e == hipSuccess && !v.cooperative) {
            v.cooperative = 1;
            e = hipGraphKernelNodeSetAttribute(nodes[k], hipKernelNodeAttributeCooperative, &v);
            if (e == hipSuccess) e = hipGraphKernelNodeGetAttribute(nodes[k], hipKernelNodeAttributeCooperative, &v);
            if (e == hipSuccess && !v.cooperative) e = hipErrorNotSupported;
        }
    }
    if (e == hipSuccess && kernels != 1) e = hipErrorInvalidValue;
    return e;
}

// Workgroups of the persistent launch: the chosen count, but no more than
// there are work items (node blocks, or wavefronts' worth of lines) for the
// instances still running, since every grid barrier costs in proportion to
// the workgroups that take part.
int batch_grid(const lbm_batch* b)
{
    const int W = b->block / 64;
    const int items = std::max(b->nblk_total, (b->nlines + W - 1) / W);
    return std::max(1, std::min(b->grid, items));
}

// One chunk as a graph: the cooperative kernel, then the status and flag
// read-backs into the pinned host buffers.  First by stream capture of the
// cooperative launch; where the runtime cannot capture it, by building the
// graph from a kernel node with the cooperative attribute.
hipError_t batch_graph(lbm_batch* b, const BatchArgs& a, hipGraphExec_t* out, std::string& how)
{
    const void* kfn = batch_kernel(b->block);
    BatchArgs aa = a;
    void* args[] = { &aa };
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t l = hipLaunchCooperativeKernel(kfn, dim3(batch_grid(b)), dim3(b->block), args, 0, b->cap_stream);
        if (l == hipSuccess)
            l = hipMemcpyAsync(b->h_st, b->d_st, sizeof(BState) * b->n, hipMemcpyDeviceToHost, b->cap_stream);
        if (l == hipSuccess)
            l = hipMemcpyAsync(b->h_flag, b->d_flag, 2 * sizeof(int), hipMemcpyDeviceToHost, b->cap_stream);
        e = hipStreamEndCapture(b->cap_stream, &g);
        if (e == hipSuccess) e = l;
        if (e == hipSuccess && !g) e = hipErrorInvalidValue;
        if (e == hipSuccess) e = ensure_cooperative(g);
        how = "graph: captured cooperative launch";
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        g = nullptr;
        const std::string first = hipGetErrorString(e);
        e = hipGraphCreate(&g, 0);
        hipGraphNode_t kn = nullptr, m1 = nullptr, m2 = nullptr;
        if (e == hipSuccess) {
            hipKernelNodeParams kp{};
            kp.func = const_cast<void*>(kfn);
            kp.gridDim = dim3(batch_grid(b));
            kp.blockDim = dim3(b->block);
            kp.sharedMemBytes = 0;
            kp.kernelParams = args;
            kp.extra = nullptr;
            e = hipGraphAddKernelNode(&kn, g, nullptr, 0, &kp);
        }
        if (e == hipSuccess) {
            hipKernelNodeAttrValue v{};
            v.cooperative = 1;
            e = hipGraphKernelNodeSetAttribute(kn, hipKernelNodeAttributeCooperative, &v);
        }
        if (e == hipSuccess)
            e = hipGraphAddMemcpyNode1D(&m1, g, &kn, 1, b->h_st, b->d_st, sizeof(BState) * b->n,
                                        hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipGraphAddMemcpyNode1D(&m2, g, &m1, 1, b->h_flag, b->d_flag, 2 * sizeof(int),
                                        hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = ensure_cooperative(g);
        how = "graph: cooperative kernel node (stream capture of the cooperative launch failed: " + first + ")";
    }
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

// The phase form of one chunk, issued on stream st: for each loop step the
// density, the chemical potential (with the compact schemes' first line
// solves), the compact schemes' second line solves, the two check kernels on
// the loop steps in `due`, and the collision; then the counters.  Every
// kernel strides over its items, so the grids only set how many workgroups
// share them: one per node-block item, per BN/64 lines, per BN instances.
template <int BN>
hipError_t batch_phases_t(const lbm_batch* b, const BatchArgs& a, const std::vector<char>& due, hipStream_t st)
{
    constexpr int W = BN / 64;
    const unsigned gi = (unsigned)std::max(1, b->nblk_total);
    const unsigned gl = (unsigned)std::max(1, (b->nlines + W - 1) / W);
    const unsigned gm = b->has_compact ? std::max(gi, gl) : gi;
    const unsigned gf = (unsigned)std::max(1, (b->n + BN - 1) / BN);
    for (int s = 0; s < a.nsteps; ++s) {
        hipLaunchKernelGGL(k_bp_density<BN>, dim3(gi), dim3(BN), 0, st, a, s);
        hipLaunchKernelGGL(k_bp_mu<BN>, dim3(gm), dim3(BN), 0, st, a);
        if (b->has_compact) hipLaunchKernelGGL(k_bp_lines1<BN>, dim3(gl), dim3(BN), 0, st, a);
        if (due[(size_t)s]) {
            hipLaunchKernelGGL(k_bp_check<BN>, dim3(gi), dim3(BN), 0, st, a, s);
            hipLaunchKernelGGL(k_bp_fold<BN>, dim3(gf), dim3(BN), 0, st, a, s);
        }
        hipLaunchKernelGGL(k_bp_collide<BN>, dim3(gi), dim3(BN), 0, st, a, s);
    }
    hipLaunchKernelGGL(k_bp_finish<BN>, dim3(gf), dim3(BN), 0, st, a);
    return hipGetLastError();
}

hipError_t batch_phases(const lbm_batch* b, const BatchArgs& a, const std::vector<char>& due, hipStream_t st)
{
    switch (b->block) {
    case 256: return batch_phases_t<256>(b, a, due, st);
    case 1024: return batch_phases_t<1024>(b, a, due, st);
    default: return batch_phases_t<512>(b, a, due, st);
    }
}

// Loop steps of the next chunk on which some instance that is still running
// is at a multiple of check_every (from the counts read back after the last
// chunk).  Instances that retire during the chunk were running at its start,
// so the set covers every check the persistent kernel would make there.
std::vector<char> batch_due(const lbm_batch* b, int todo, int check_every)
{
    std::vector<char> due((size_t)todo, 0);
    for (int i = 0; i < b->n; ++i) {
        const BState& S = b->h_st[i];
        if (S.status != B_RUNNING) continue;
        long long s = (check_every - S.steps % check_every) % check_every;
        for (; s < todo; s += check_every) due[(size_t)s] = 1;
    }
    return due;
}

// One chunk of the phase form as a graph (stream capture), with the status
// and flag read-backs.
hipError_t batch_phase_graph(lbm_batch* b, const BatchArgs& a, const std::vector<char>& due, hipGraphExec_t* out)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t l = batch_phases(b, a, due, b->cap_stream);
    if (l == hipSuccess)
        l = hipMemcpyAsync(b->h_st, b->d_st, sizeof(BState) * b->n, hipMemcpyDeviceToHost, b->cap_stream);
    if (l == hipSuccess) l = hipMemcpyAsync(b->h_flag, b->d_flag, 2 * sizeof(int), hipMemcpyDeviceToHost, b->cap_stream);
    e = hipStreamEndCapture(b->cap_stream, &g);
    if (e == hipSuccess) e = l;
    if (e == hipSuccess && !g) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(const lbm_params* ps, int n)
{
    if (!ps || n < 1) return 0;
    BatchLayout B;
    const char* why = nullptr;
    if (!batch_layout(ps, n, B, &why)) return 0;
    return B.total;
}

int lbm_batch_init(const lbm_params* ps, const double* const* rho0s, int n, void* d_workspace, size_t ws_bytes,
                   void* hip_stream, lbm_batch** out)
{
    if (!out) return bfail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ps || !rho0s || n < 1) return bfail(nullptr, LBM_EINVAL, "bad batch arguments");
    BatchLayout B;
    const char* why = nullptr;
    if (!batch_layout(ps, n, B, &why)) return bfail(nullptr, LBM_EINVAL, why);
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
        return bfail(nullptr, LBM_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < B.total) return bfail(nullptr, LBM_ENOSPC, "batch workspace too small");
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(nullptr, LBM_EHIP, "out of host memory");
    b->n = n;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->ws = static_cast<char*>(d_workspace);
    b->ctx.assign(n, nullptr);
    b->inst.resize(n);
    b->use_graph = std::getenv("LBM_NO_GRAPH") == nullptr;
    int rc = LBM_OK;
    for (int i = 0; i < n && rc == LBM_OK; ++i) {
        lbm_ctx* c = nullptr;
        const size_t sz = layout_of(&ps[i]).total;
        rc = lbm_init(&ps[i], rho0s[i], 0, b->ws + B.inst_off[i], sz, hip_stream, &c);
        if (rc != LBM_OK) { b->err = "instance " + std::to_string(i) + ": " + g_thread_error; break; }
        c->fused = false;
        c->in_batch = true;
        drop_branches(c);     // instances are stepped by the batched kernel
        b->ctx[i] = c;
        BInst& I = b->inst[i];
        I.g = c->g;
        I.scheme = ps[i].scheme;
        I.rx = c->rx;
        I.eos = c->eos;
        I.S[0] = c->S[0]; I.S[1] = c->S[1];
        I.rho = c->rhob[0]; I.mu = c->mu;
        I.grho = c->grho; I.gmu = c->gmu; I.lap = c->lap; I.wtmp = c->wtmp;
        I.cc = compact_scheme(ps[i].scheme);
        I.z = c->z; I.zscale = c->zscale;
        I.K = c->lines[0].K;
    }
    if (rc != LBM_OK) { std::string e = b->err; lbm_batch_free(b); return bfail(nullptr, rc, e); }
    size_t off = B.tables;
    b->d_inst = reinterpret_cast<BInst*>(b->ws + off); off = align_up(off + sizeof(BInst) * n);
    b->d_st = reinterpret_cast<BState*>(b->ws + off); off = align_up(off + sizeof(BState) * n);
    b->d_blk_inst = reinterpret_cast<int*>(b->ws + off); off = align_up(off + sizeof(int) * B.nblk);
    b->d_partial = reinterpret_cast<double*>(b->ws + off); off = align_up(off + sizeof(double) * B.nblk);
    b->d_lines = reinterpret_cast<BLine*>(b->ws + off); off = align_up(off + sizeof(BLine) * std::max(1, B.nlines));
    b->d_flag = reinterpret_cast<int*>(b->ws + off);
    // the grid lines of the compact-scheme instances, rows then columns; lines
    // of at most kShortLine points go 64 to an item (one per lane)
    std::vector<BLine> lines;
    for (int i = 0; i < n; ++i) {
        if (!is_compact(ps[i].scheme)) continue;
        for (int axis = 0; axis < 2; ++axis) {
            const int len = axis == 0 ? ps[i].nx : ps[i].ny, count = axis == 0 ? ps[i].ny : ps[i].nx;
            const int per = len <= kShortLine ? 64 : 1;
            for (int j = 0; j < count; j += per) lines.push_back(BLine{ i, axis, j, std::min(per, count - j) });
        }
    }
    b->all_lines = lines;
    std::vector<BState> st(n);
    for (auto& x : st) { x.status = B_RUNNING; x.steps = 0; x.stop = -1; x.U = 0.0; x.U_prev = 0.0; }
    static const int zero[2] = { 0, 0 };
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&b->h_st), sizeof(BState) * n, hipHostMallocDefault);
    if (e == hipSuccess) std::memcpy(b->h_st, st.data(), sizeof(BState) * n);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->h_flag), 2 * sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) b->h_flag[0] = b->h_flag[1] = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_st, st.data(), sizeof(BState) * n, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_flag, zero, 2 * sizeof(int), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = batch_tables(b);
    int dev = 0, ncu = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    for (int k = 0; k < kNumBatchBlocks && e == hipSuccess; ++k) {
        int per_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel(kBatchBlocks[k]), kBatchBlocks[k], 0);
        b->max_grid_of[k] = std::max(1, per_cu * ncu);
    }
    if (e == hipSuccess && b->use_graph) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        std::string m = std::string("batch setup: ") + hipGetErrorString(e);
        lbm_batch_free(b);
        return bfail(nullptr, LBM_EHIP, m);
    }
    b->grid = b->max_grid_of[batch_block_index(b->block)];
    *out = b;
    return LBM_OK;
}

int lbm_batch_set_grid(lbm_batch* b, int workgroups)
{
    if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
    if (workgroups < 1 || workgroups > lbm_batch_max_grid(b)) return bfail(b, LBM_EINVAL, "workgroups out of range");
    b->grid = workgroups;
    return LBM_OK;
}

int lbm_batch_max_grid(const lbm_batch* b) { return b ? b->max_grid_of[batch_block_index(b->block)] : 0; }

int lbm_batch_set_block(lbm_batch* b, int nodes)
{
    if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
    const int k = batch_block_index(nodes);
    if (k < 0) return bfail(b, LBM_EINVAL, "block must be 256, 512 or 1024 nodes");
    if (nodes == b->block) return LBM_OK;
    b->block = nodes;
    const hipError_t e = batch_tables(b);
    if (e != hipSuccess) return bfail(b, LBM_EHIP, std::string("batch tables: ") + hipGetErrorString(e));
    b->grid = b->max_grid_of[k];
    return LBM_OK;
}

int lbm_batch_block(const lbm_batch* b) { return b ? b->block : 0; }

int lbm_batch_set_form(lbm_batch* b, int form)
{
    if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
    if (form != LBM_BATCH_PERSISTENT && form != LBM_BATCH_PHASES)
        return bfail(b, LBM_EINVAL, "form must be LBM_BATCH_PERSISTENT or LBM_BATCH_PHASES");
    b->form = form;
    return LBM_OK;
}

int lbm_batch_form(const lbm_batch* b) { return b ? b->form : -1; }

const char* lbm_batch_launch_mode(const lbm_batch* b) { return b ? b->mode.c_str() : ""; }

int lbm_batch_run(lbm_batch* b, long nsteps, long check_every, double tol, long chunk, int* status, long* steps,
                  double* umax)
{
    if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
    if (nsteps < 0 || check_every < 1 || chunk < 1 || chunk > (1L << 30) || check_every > (1L << 30) ||
        !(tol >= 0.0))
        return bfail(b, LBM_EINVAL, "bad run arguments");
    long done = 0;
    bool ran = false;
    while (done < nsteps) {
        {
            // instances retired since the tables were built: tables of the
            // running ones (the graphs hold the old item counts, so they go)
            int running = 0;
            for (int i = 0; i < b->n; ++i) running += b->h_st[i].status == B_RUNNING;
            if (running == 0) break;
            if (running < b->table_running) {
                const hipError_t te = batch_tables(b);
                if (te != hipSuccess) return bfail(b, LBM_EHIP, std::string("batch tables: ") + hipGetErrorString(te));
                drop_graphs(b);
            }
        }
        // the phase form issues about four launches per step, so its chunks
        // (and the graphs that hold them) are capped at kPhaseChunk steps
        const long todo = std::min(b->form == LBM_BATCH_PHASES ? std::min(chunk, kPhaseChunk) : chunk, nsteps - done);
        BatchArgs a;
        a.inst = b->d_inst; a.st = b->d_st; a.ninst = b->n;
        a.nblk_total = b->nblk_total;
        a.blk_inst = b->d_blk_inst;
        a.partial = b->d_partial;
        a.has_compact = b->has_compact;
        a.lines = b->d_lines;
        a.nlines = b->nlines;
        a.nsteps = (int)todo;
        a.check_every = (int)check_every;
        a.tol = tol;
        a.not_cooperative = b->d_flag;
        a.launches = reinterpret_cast<unsigned*>(b->d_flag + 1);
        hipError_t e = hipSuccess;
        bool replayed = false;
        const bool phases = b->form == LBM_BATCH_PHASES;
        const std::vector<char> due = phases ? batch_due(b, (int)todo, (int)check_every) : std::vector<char>();
        if (b->use_graph) {
            lbm_batch::Graph* gr = nullptr;
            for (auto& g : b->graphs)
                if (g.form == b->form && g.todo == (int)todo && g.check == (int)check_every && g.tol == tol &&
                    g.grid == (phases ? 0 : batch_grid(b)) && g.block == b->block && g.due == due)
                    gr = &g;
            if (!gr) {
                // a bounded cache: chunk lengths and check intervals that do
                // not align give one phase graph per offset of the checks
                if (b->graphs.size() >= kMaxBatchGraphs) drop_graphs(b);
                hipGraphExec_t ex = nullptr;
                std::string how = "graph: captured phase kernels";
                const hipError_t ge = phases ? batch_phase_graph(b, a, due, &ex) : batch_graph(b, a, &ex, how);
                if (ge == hipSuccess) {
                    b->graphs.push_back({ b->form, (int)todo, (int)check_every, phases ? 0 : batch_grid(b), b->block, tol,
                                          due, ex, how });
                    gr = &b->graphs.back();
                } else {
                    (void)hipGetLastError();
                    b->use_graph = false;
                    b->mode = std::string(phases ? "plain phase kernels" : "plain cooperative launches") +
                              " (no graph: " + hipGetErrorString(ge) + ")";
                }
            }
            if (gr) {
                b->mode = gr->how;
                e = hipGraphLaunch(gr->exec, b->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
                if (e == hipSuccess && (b->h_flag[0] || (unsigned)b->h_flag[1] != b->launches + 1)) {
                    // the replay did not launch cooperatively (the kernel
                    // returned at once) or did not run the kernels to their
                    // end: no step was taken, so this chunk runs again below
                    static const int zero = 0;
                    e = hipMemcpyAsync(b->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice, b->stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
                    b->h_flag[0] = 0;
                    drop_graphs(b);
                    b->use_graph = false;
                    b->mode = std::string(phases ? "plain phase kernels" : "plain cooperative launches") +
                              " (a graph replay did not run the kernels)";
                } else if (e == hipSuccess) {
                    b->launches++;
                    replayed = true;
                }
            }
        }
        if (e == hipSuccess && !replayed && !phases) {
            if (b->mode.rfind("plain cooperative launches", 0) != 0) b->mode = "plain cooperative launches";
            void* args[] = { &a };
            e = hipLaunchCooperativeKernel(batch_kernel(b->block), dim3(batch_grid(b)), dim3(b->block), args, 0,
                                           b->stream);
            if (e != hipSuccess) {
                // this runtime refuses cooperative launches while another
                // process holds the device: the chunk runs as phase kernels
                // (bitwise the same steps), and so do the later ones
                b->mode = std::string("plain phase kernels (the cooperative launch was refused: ") +
                          hipGetErrorString(e) + ")";
                (void)hipGetLastError();
                e = hipSuccess;
                b->form = LBM_BATCH_PHASES;
                b->use_graph = false;
                drop_graphs(b);
                a.nsteps = (int)std::min(todo, kPhaseChunk);   // the phase form's launch sequences stay bounded
            } else {
                e = hipMemcpyAsync(b->h_st, b->d_st, sizeof(BState) * b->n, hipMemcpyDeviceToHost, b->stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(b->h_flag, b->d_flag, 2 * sizeof(int), hipMemcpyDeviceToHost, b->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
                if (e == hipSuccess && (b->h_flag[0] || (unsigned)b->h_flag[1] != b->launches + 1)) {
                    // the kernel found no grid barrier and returned at once, or
                    // did not run: no step of this launch was taken
                    static const int zero = 0;
                    b->h_flag[0] = 0;
                    (void)hipMemcpyAsync(b->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice, b->stream);
                    (void)hipStreamSynchronize(b->stream);
                    return bfail(b, LBM_EHIP, "the runtime did not run the batch kernel as a cooperative launch "
                                              "(no grid barrier, or no run); no step was taken");
                }
                if (e == hipSuccess) {
                    b->launches++;
                    replayed = true;
                }
            }
        }
        if (e == hipSuccess && !replayed) {
            // the phase form without a graph (also the fallback above)
            if (b->mode.rfind("plain phase kernels", 0) != 0) b->mode = "plain phase kernels";
            const std::vector<char> d = batch_due(b, a.nsteps, (int)check_every);
            e = batch_phases(b, a, d, b->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(b->h_st, b->d_st, sizeof(BState) * b->n, hipMemcpyDeviceToHost, b->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(b->h_flag, b->d_flag, 2 * sizeof(int), hipMemcpyDeviceToHost, b->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
            if (e == hipSuccess && (unsigned)b->h_flag[1] != b->launches + 1)
                return bfail(b, LBM_EHIP, "the batch phase kernels did not run to their end");
            if (e == hipSuccess) b->launches++;
        }
        if (e != hipSuccess) {
            // the error is returned, not left for the caller's next runtime
            // call
            (void)hipGetLastError();
            return bfail(b, LBM_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
        }
        ran = true;
        done += a.nsteps;
        bool running = false;
        for (int i = 0; i < b->n; ++i) running |= b->h_st[i].status == B_RUNNING;
        if (!running) break;
    }
    if (!ran) {
        // no step asked for: report the current state
        const hipError_t e = hipMemcpyAsync(b->h_st, b->d_st, sizeof(BState) * b->n, hipMemcpyDeviceToHost, b->stream);
        if (e != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess)
            return bfail(b, LBM_EHIP, "batch status copy");
    }
    for (int i = 0; i < b->n; ++i) {
        lbm_ctx* c = b->ctx[i];
        c->steps = (long)b->h_st[i].steps;
        c->cur = (int)(b->h_st[i].steps & 1);
        if (status) status[i] = b->h_st[i].status;
        if (steps) steps[i] = (long)b->h_st[i].steps;
        if (umax) umax[i] = b->h_st[i].U;
    }
    return LBM_OK;
}

lbm_ctx* lbm_batch_instance(lbm_batch* b, int i)
{
    if (!b || i < 0 || i >= b->n) return nullptr;
    return b->ctx[i];
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : g_thread_error.c_str(); }

void lbm_batch_free(lbm_batch* b)
{
    if (!b) return;
    drop_graphs(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->h_st) (void)hipHostFree(b->h_st);
    if (b->h_flag) (void)hipHostFree(b->h_flag);
    for (auto* c : b->ctx) lbm_free(c);
    delete b;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned initialiser (FP32 network kernels)
// ---------------------------------------------------------------------------
extern "C" {

int mlp_param_count(void) { return MP; }

int mlp_forward(const float* d_params, const float* d_x, int B, float* d_y, float* d_acts, void* stream)
{
    if (!d_params || !d_x || !d_y || B < 1) return fail(nullptr, LBM_EINVAL, "mlp_forward: bad arguments");
    hipLaunchKernelGGL(k_mlp_fwd, dim3((B + MB - 1) / MB), dim3(MB), 0, reinterpret_cast<hipStream_t>(stream),
                       d_params, d_x, B, d_y, d_acts);
    return hip_check(nullptr, hipGetLastError(), "mlp_forward");
}

int mlp_loss_grad(const float* d_y, const float* d_t, int B, float* d_dy, float* d_loss_partial, void* stream)
{
    if (!d_y || !d_t || !d_dy || !d_loss_partial || B < 1) return fail(nullptr, LBM_EINVAL, "mlp_loss_grad: bad arguments");
    hipLaunchKernelGGL(k_mlp_loss, dim3((B + MB - 1) / MB), dim3(MB), 0, reinterpret_cast<hipStream_t>(stream),
                       d_y, d_t, B, d_dy, d_loss_partial);
    return hip_check(nullptr, hipGetLastError(), "mlp_loss_grad");
}

int mlp_backward(const float* d_params, const float* d_x, const float* d_acts, const float* d_dy, int B,
                 float* d_grad, float* d_gpart, void* stream)
{
    if (!d_params || !d_x || !d_acts || !d_dy || !d_grad || !d_gpart || B < 1)
        return fail(nullptr, LBM_EINVAL, "mlp_backward: bad arguments");
    const int nb = (B + MB - 1) / MB;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_mlp_bwd, dim3(nb), dim3(MB), 0, st, d_params, d_x, d_acts, d_dy, B, d_gpart);
    hipLaunchKernelGGL(k_mlp_gsum, dim3((MP + 255) / 256), dim3(256), 0, st, d_gpart, nb, d_grad);
    return hip_check(nullptr, hipGetLastError(), "mlp_backward");
}

int mlp_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, int step, float lr, float b1, float b2,
             float eps, void* stream)
{
    if (!d_params || !d_grad || !d_m || !d_v || step < 1) return fail(nullptr, LBM_EINVAL, "mlp_adam: bad arguments");
    const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((MP + 255) / 256), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), d_params,
                       d_grad, d_m, d_v, lr, b1, b2, eps, c1, c2);
    return hip_check(nullptr, hipGetLastError(), "mlp_adam");
}

int mlp_field(const float* d_params, const float* norm7, const lbm_params* p, double cx, double cy, double cz,
              double R, const float* feat3, double rho_g, double rho_l, double* d_rho, void* stream)
{
    if (!d_params || !norm7 || !feat3 || !d_rho) return fail(nullptr, LBM_EINVAL, "mlp_field: bad arguments");
    if (const char* why = validate(p)) return fail(nullptr, LBM_EINVAL, why);
    Grid g{};
    g.nx = p->nx; g.ny = p->ny; g.nz = p->nz;
    g.nxy = (long long)p->nx * p->ny;
    g.N = g.nxy * p->nz;
    g.ps = g.N;
    MlpNorm nm = { norm7[0], norm7[1], norm7[2], norm7[3], norm7[4], norm7[5], norm7[6] };
    hipLaunchKernelGGL(k_mlp_field, dim3((unsigned)((g.N + MB - 1) / MB)), dim3(MB), 0,
                       reinterpret_cast<hipStream_t>(stream), d_params, nm, g, cx, cy, cz, R, feat3[0], feat3[1],
                       feat3[2], rho_g, rho_l, d_rho);
    return hip_check(nullptr, hipGetLastError(), "mlp_field");
}

size_t lbm_sum_scratch_bytes(long n) { return n < 1 ? 0 : sizeof(double) * (2 * ((n + 255) / 256) + 2); }

int lbm_sum(const double* d_x, long n, double* d_scratch, double* h_sum, void* stream)
{
    if (!d_x || !d_scratch || !h_sum || n < 1) return fail(nullptr, LBM_EINVAL, "lbm_sum: bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const long long nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)nb), dim3(256), 0, st, d_x, (long long)n, d_scratch);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, st, d_scratch, nb, d_scratch + 2 * nb);
    double h[2];
    int r = hip_check(nullptr, hipMemcpyAsync(h, d_scratch + 2 * nb, sizeof(h), hipMemcpyDeviceToHost, st), "sum copy");
    if (r) return r;
    r = hip_check(nullptr, hipStreamSynchronize(st), "sum sync");
    if (r) return r;
    *h_sum = h[1];
    return LBM_OK;
}

int lbm_interface_mass(double* d_rho, long n, double rho_g, double rho_l, double target_mass, double* d_scratch,
                       void* stream)
{
    if (!d_rho || !d_scratch || n < 1 || !(rho_l > rho_g) || !std::isfinite(rho_g) || !std::isfinite(rho_l) ||
        !std::isfinite(target_mass))
        return fail(nullptr, LBM_EINVAL, "lbm_interface_mass: bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const long long nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_mass_partials, dim3((unsigned)nb), dim3(256), 0, st, d_rho, (long long)n, rho_g, rho_l,
                       d_scratch);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(1024), 0, st, d_scratch, nb, d_scratch + 2 * nb);
    hipLaunchKernelGGL(k_mass_apply, dim3((unsigned)nb), dim3(256), 0, st, d_rho, (long long)n, rho_g, rho_l,
                       d_scratch + 2 * nb, target_mass);
    return hip_check(nullptr, hipGetLastError(), "lbm_interface_mass");
}

// lbm_sum_static: the deterministic sum with its scratch (the per-workgroup
// partials of k_sum_partials and the two results of k_reduce_final) in a
// fixed device array, for callers that cannot allocate.
size_t lbm_sum_static_max(void) { return (size_t)kStaticSumMaxN; }

int lbm_sum_static(const double* d_x, long n, double* h_sum, void* stream)
{
    if (!d_x || !h_sum || n < 1) return fail(nullptr, LBM_EINVAL, "lbm_sum_static: bad arguments");
    if ((long long)n > kStaticSumMaxN)
        return fail(nullptr, LBM_EINVAL, "lbm_sum_static: n = " + std::to_string(n) + " exceeds the maximum " +
                                             std::to_string(kStaticSumMaxN) + " of the static scratch");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double* ws = nullptr;
    int r = static_sum_scratch(st, &ws);
    if (r) return r;
    const long long nb = (n + 255) / 256;
    // every partial the final reduction reads is written first: nothing needs clearing
    hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)nb), dim3(256), 0, st, d_x, (long long)n, ws);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, st, ws, nb, ws + 2 * nb);
    r = hip_check(nullptr, hipGetLastError(), "lbm_sum_static launch");
    if (r) return r;
    double h[2];
    r = hip_check(nullptr, hipMemcpyAsync(h, ws + 2 * nb, sizeof(h), hipMemcpyDeviceToHost, st), "sum copy");
    if (r) return r;
    r = hip_check(nullptr, hipStreamSynchronize(st), "sum sync");
    if (r) return r;
    *h_sum = h[1];
    return LBM_OK;
}

int lbm_probe_copy(int lattice, int nx, int ny, int nz, const double* d_src, double* d_dst, int pull, void* stream)
{
    if (!d_src || !d_dst || (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) || nx < 1 || ny < 1 || nz < 1 ||
        (lattice == LBM_D2Q9 && nz != 1))
        return fail(nullptr, LBM_EINVAL, "lbm_probe_copy: bad arguments");
    if ((long long)nx * ny * nz > (1LL << 38))   // keeps the launch's workgroup count within 32 bits
        return fail(nullptr, LBM_EINVAL, "lbm_probe_copy: grid too large");
    Grid g{};
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.nxy = (long long)nx * ny;
    g.N = g.nxy * nz;
    g.ps = g.N;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid(blocks_for(g.N, 256)), block(256);
    if (lattice == LBM_D3Q19) {
        if (pull) hipLaunchKernelGGL((k_probe_copy<1, true>), grid, block, 0, st, d_src, d_dst, g);
        else hipLaunchKernelGGL((k_probe_copy<1, false>), grid, block, 0, st, d_src, d_dst, g);
    } else {
        if (pull) hipLaunchKernelGGL((k_probe_copy<0, true>), grid, block, 0, st, d_src, d_dst, g);
        else hipLaunchKernelGGL((k_probe_copy<0, false>), grid, block, 0, st, d_src, d_dst, g);
    }
    return hip_check(nullptr, hipGetLastError(), "lbm_probe_copy");
}

}  // extern "C"
