// lbm_batch.hpp -- batched sweep: many uneven D2Q9 instances (droplets and flat
// slabs at different temperatures, radii and schemes) advanced together, by
// one cooperative persistent kernel or by one ordinary launch per phase.
//
// Every instance keeps its own populations, density and chemical potential in
// one pool.  A step is a fixed sequence of phases (density; the chemical
// potential of the explicit schemes together with the compact schemes' line
// solves of D rho and D(D rho); the compact schemes' line solves of D mu_hat;
// collision); within a phase the workgroups stride over the work items of all
// running instances.  In the persistent form a grid-wide barrier separates the
// phases: the cooperative launch guarantees that every workgroup is resident,
// every workgroup executes the same phase sequence, and every loop is bounded,
// so the barriers always complete.  In the phase form each phase is a launch
// of its own and the kernel boundary separates them.
// Every check_every steps the spurious current U = max |v| of each instance is
// reduced (fixed order) and compared with the previous check: an instance
// whose U changed by less than tol is CONVERGED, one with a non-finite state
// or U above the sound speed is DIVERGED; both stop stepping.
// During a launch the step count of an instance stays at its launch-start
// value (loop step s is its step steps + s), so no phase of the step is spent
// on counters; the counts advance once, after the loop.  The check phase and
// its two barriers (or two launches) run only on loop steps where some
// instance is due.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>
#include "lbm_kernels.hpp"

namespace lbm {

enum BatchStatus { B_RUNNING = 0, B_CONVERGED = 1, B_DIVERGED = 2 };

struct BInst {
    Grid g;
    int scheme;
    Relax rx;
    Eos eos;
    double *S[2], *rho, *mu, *grho, *gmu, *lap, *wtmp;
    Compact cc;
    double z, zscale;
    int K;                  // warm-up of the compact recursions, |z|^K < 1e-18
    int blk0, nblk;         // node-block items [blk0, blk0 + nblk)
    int part0;              // first partial slot of its node blocks
};

struct BState {             // per instance, updated by the kernel
    int status;
    long long steps;        // steps taken; fixed during a launch, advanced at its end
    long long stop;         // loop step of a launch at which the instance retired, else -1
    double U, U_prev;
};

// Node-block sizes of the batched kernel: nodes per node-block item (one per
// thread) and threads per workgroup.  A tuner picks one with the workgroup
// count; 512 is the default.
constexpr int kBatchBlocks[] = { 256, 512, 1024 };
constexpr int kNumBatchBlocks = 3;
constexpr int kBatchDefaultBlock = 512;
constexpr int kBatchMinBlock = 256;

// ---------------------------------------------------------------------------
// per-node bodies with runtime scheme dispatch
// ---------------------------------------------------------------------------
template <int SCH>
__device__ void b_mu_node(const BInst& I, long long n, int x, int y)
{
    constexpr int R = radius(SCH);
    Nbr<R, 2> nb(x, y, 0, I.g);
    I.mu[n] = mu_bulk(I.rho[n], I.eos) - I.eos.kappa * lap_at<2, SCH, R>(I.rho, nb);
}

template <int SCH>
__device__ void b_force(const BInst& I, long long n, int x, int y, double r, double& Fx, double& Fy, double& Fz)
{
    force_at<0, SCH>(I.rho, I.mu, I.grho, I.gmu, I.g, n, x, y, 0, r, Fx, Fy, Fz);
}

__device__ void b_force_any(const BInst& I, long long n, int x, int y, double r, double& Fx, double& Fy, double& Fz)
{
    switch (I.scheme) {
    case CD2: b_force<CD2>(I, n, x, y, r, Fx, Fy, Fz); break;
    case CD4: b_force<CD4>(I, n, x, y, r, Fx, Fy, Fz); break;
    case CD6: b_force<CD6>(I, n, x, y, r, Fx, Fy, Fz); break;
    case E4: b_force<E4>(I, n, x, y, r, Fx, Fy, Fz); break;
    case E6: b_force<E6>(I, n, x, y, r, Fx, Fy, Fz); break;
    case E8: b_force<E8>(I, n, x, y, r, Fx, Fy, Fz); break;
    case E10: b_force<E10>(I, n, x, y, r, Fx, Fy, Fz); break;
    default: b_force<OCFDS4>(I, n, x, y, r, Fx, Fy, Fz); break;   // gradient fields
    }
}

__device__ void b_moments(const BInst& I, const double* S, long long n, int x, int y, double (&f)[9], double& r,
                          double& jx, double& jy)
{
    using L = Lat<0>;
    (void)n;
    Nbr<1, 2> nb(x, y, 0, I.g);
    r = jx = jy = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        f[i] = S[(long long)i * I.g.ps + nb.at(-L::ex(i), -L::ey(i), 0)];
        r += f[i];
        jx += L::ex(i) * f[i];
        jy += L::ey(i) * f[i];
    }
}

// One grid line of a compact-scheme instance: along x (axis 0, line = row y)
// or along y (axis 1, line = column x).
// A work item of the line stages: cnt = 1 is one line (idx) solved by a
// wavefront; cnt > 1 is the cnt consecutive lines idx .. idx + cnt - 1 (cnt <=
// 64) of at most kShortLine points, one per lane.
struct BLine {
    int inst, axis, idx, cnt;
};
constexpr int kShortLine = 16;

// Compact derivative (Eq 21) of one short periodic line (4 <= n <= kShortLine)
// by one thread: both recursions from a zero start, each closed around the
// line exactly (the value entering the line is the local end / (1 - z^n)).
template <class Load>
__device__ void thread_line(const BInst& I, Load&& ld, double* __restrict__ out, long long base, long long sa, int n)
{
    const double ha = 0.5 * I.cc.ca, hb = 0.25 * I.cc.cb, hc = I.cc.cc / 6.0, z = I.z;
    double r[kShortLine + 6];
#pragma unroll
    for (int k = 0; k < kShortLine + 6; ++k) {
        int idx = k - 3;                    // in [-3, n + 2]; n >= 4
        idx += idx < 0 ? n : 0;
        idx -= idx >= n ? n : 0;
        r[k] = k < n + 6 ? ld(base + idx * sa) : 0.0;
    }
    double acc = 0.0, pz = 1.0;
#pragma unroll
    for (int i = 0; i < kShortLine; ++i) {
        if (i < n) {
            acc = ha * (r[i + 4] - r[i + 2]) + hb * (r[i + 5] - r[i + 1]) + hc * (r[i + 6] - r[i]) + z * acc;
            r[i] = acc;
            pz *= z;
        }
    }
    const double T = acc / (1.0 - pz);
    double q = z;
#pragma unroll
    for (int i = 0; i < kShortLine; ++i)
        if (i < n) { r[i] += q * T; q *= z; }
    acc = 0.0;
#pragma unroll
    for (int i = kShortLine - 1; i >= 0; --i)
        if (i < n) { acc = r[i] + z * acc; r[i] = acc; }
    const double U = acc / (1.0 - pz);
    q = z;
#pragma unroll
    for (int i = kShortLine - 1; i >= 0; --i)
        if (i < n) { out[base + i * sa] = I.zscale * (r[i] + q * U); q *= z; }
}

// Compact derivative (Eq 21) along one periodic line of instance I of the
// field that ld(o) reads, into out, by one wavefront (wave_line).
template <class Load>
__device__ void b_line(const BInst& I, Load&& ld, double* __restrict__ out, long long base, long long sa, int n,
                       int lane)
{
    double y[kLineSeg];
    int s0, Ll;
    wave_line(ld, base, sa, n, lane, I.cc, I.z, I.zscale, y, s0, Ll);
#pragma unroll
    for (int i = 0; i < kLineSeg; ++i)
        if (i < Ll) out[base + (s0 + i) * sa] = y[i];
}

struct BatchArgs {
    BInst* inst;
    BState* st;
    int ninst;
    int nblk_total;           // node-block items over all instances
    int* blk_inst;            // node-block item -> instance
    double* partial;          // one max |v| per node-block item
    int has_compact;
    const BLine* lines;       // the grid lines of every compact-scheme instance
    int nlines;
    int nsteps;
    int check_every;
    double tol;
    int* not_cooperative;     // set (and nothing else done) if the launch was not cooperative
    unsigned* launches;       // completed launches: one more at the end of each
};

// ---------------------------------------------------------------------------
// The phases of loop step s of a launch.  Each strides over its work items
// from `first` by `stride` (node-block items per workgroup, lines per
// wavefront, instances per thread), so that one body serves both launch
// forms: the persistent kernel (every workgroup runs every phase, grid
// barriers between them) and the phase kernels (one launch per phase, the
// kernel boundary as the barrier).
// ---------------------------------------------------------------------------

// density of the current state
template <int BNODES>
__device__ void bp_density(const BatchArgs& a, int s, int first, int stride)
{
    for (int it = first; it < a.nblk_total; it += stride) {
        const int ii = a.blk_inst[it];
        const BInst& I = a.inst[ii];
        if (a.st[ii].status != B_RUNNING) continue;
        const double* Sc = I.S[(a.st[ii].steps + s) & 1];
        const long long n = (long long)(it - I.blk0) * BNODES + threadIdx.x;
        if (n < I.g.N) {
            int x, y, z;
            coords(n, I.g, x, y, z);
            double f[9], r, jx, jy;
            b_moments(I, Sc, n, x, y, f, r, jx, jy);
            I.rho[n] = r;
        }
    }
}

// Compact schemes: the line solves.  One wavefront takes a line (the item is
// uniform over the wavefront); the x and y lines of a stage run together.
// Stage 0 solves D rho and then, from the values it has just written (its own
// line only), D(D rho); stage 1 solves D mu_hat with mu_hat = k^2 psi'(rho) -
// kappa_hat (D_x D_x rho + D_y D_y rho) formed as it is read (Eq 16; the
// Laplacian terms in axis order), so mu_hat is never stored: the force of the
// compact schemes takes only the gradients.  first/stride count wavefronts.
template <int BNODES>
__device__ void bp_lines(const BatchArgs& a, int stage, int first, int stride)
{
    const int lane = threadIdx.x % 64;
    for (int t = first; t < a.nlines; t += stride) {
        const BLine ln = a.lines[t];
        if (a.st[ln.inst].status != B_RUNNING) continue;
        const BInst& I = a.inst[ln.inst];
        const long long N = I.g.N;
        const long long sa = ln.axis == 0 ? 1 : I.g.nx;
        const int n = ln.axis == 0 ? I.g.nx : I.g.ny;
        // the line of this wavefront, or of this lane for a packed item
        const int li = ln.idx + (ln.cnt > 1 ? lane : 0);
        const long long base = ln.axis == 0 ? (long long)li * I.g.nx : li;
        const double* rho = I.rho;
        const double* lap = I.lap;
        auto mu_at = [&](long long o) {
            return mu_bulk(rho[o], I.eos) - I.eos.kappa * (lap[o] + lap[N + o]);
        };
        if (ln.cnt > 1) {
            if (lane < ln.cnt) {
                if (stage == 0) {
                    double* g1 = I.grho + ln.axis * N;
                    thread_line(I, [&](long long o) { return rho[o]; }, g1, base, sa, n);
                    __threadfence_block();   // the stores above before the loads below
                    thread_line(I, [&](long long o) { return g1[o]; }, I.lap + ln.axis * N, base, sa, n);
                } else {
                    thread_line(I, mu_at, I.gmu + ln.axis * N, base, sa, n);
                }
            }
        } else if (stage == 0) {
            double* g1 = I.grho + ln.axis * N;
            b_line(I, [&](long long o) { return rho[o]; }, g1, base, sa, n, lane);
            __threadfence_block();   // this wavefront's stores before its loads
            b_line(I, [&](long long o) { return g1[o]; }, I.lap + ln.axis * N, base, sa, n, lane);
        } else {
            b_line(I, mu_at, I.gmu + ln.axis * N, base, sa, n, lane);
        }
    }
}

// chemical potential of the explicit schemes
template <int BNODES>
__device__ void bp_mu(const BatchArgs& a, int first, int stride)
{
    for (int it = first; it < a.nblk_total; it += stride) {
        const int ii = a.blk_inst[it];
        const BInst& I = a.inst[ii];
        if (a.st[ii].status != B_RUNNING || is_compact(I.scheme)) continue;
        const long long n = (long long)(it - I.blk0) * BNODES + threadIdx.x;
        if (n < I.g.N) {
            int x, y, z;
            coords(n, I.g, x, y, z);
            switch (I.scheme) {
            case CD2: b_mu_node<CD2>(I, n, x, y); break;
            case CD4: b_mu_node<CD4>(I, n, x, y); break;
            case CD6: b_mu_node<CD6>(I, n, x, y); break;
            case E4: b_mu_node<E4>(I, n, x, y); break;
            case E6: b_mu_node<E6>(I, n, x, y); break;
            case E10: b_mu_node<E10>(I, n, x, y); break;
            default: b_mu_node<E8>(I, n, x, y); break;
            }
        }
    }
}

// some instance is at a multiple of check_every at loop step s (the same
// answer in every workgroup, from the launch-start counts)
template <int BNODES>
__device__ bool bp_due(const BatchArgs& a, int s)
{
    int due = 0;
    for (int i = threadIdx.x; i < a.ninst; i += BNODES) due |= (a.st[i].steps + s) % a.check_every == 0;
    return __syncthreads_or(due);
}

// convergence check, first half: max |v| of every node-block item of an
// instance that is due, reduced in a fixed order
template <int BNODES>
__device__ void bp_check_partials(const BatchArgs& a, int s, int first, int stride, double* red)
{
    for (int it = first; it < a.nblk_total; it += stride) {
        const int ii = a.blk_inst[it];
        if (a.st[ii].status != B_RUNNING || (a.st[ii].steps + s) % a.check_every != 0) continue;
        const BInst& I = a.inst[ii];
        const double* Sc = I.S[(a.st[ii].steps + s) & 1];
        const long long n = (long long)(it - I.blk0) * BNODES + threadIdx.x;
        double vm = 0.0;
        if (n < I.g.N) {
            int x, y, z;
            coords(n, I.g, x, y, z);
            double f[9], r, jx, jy, Fx, Fy, Fz;
            b_moments(I, Sc, n, x, y, f, r, jx, jy);
            b_force_any(I, n, x, y, r, Fx, Fy, Fz);
            const double ir = 1.0 / r;
            const double vx = (jx + 0.5 * Fx) * ir, vy = (jy + 0.5 * Fy) * ir;
            vm = sqrt(vx * vx + vy * vy);
            if (!(r == r) || r - r != 0.0) vm = r - r;
        }
        for (int o = 32; o > 0; o >>= 1) vm = nmax(vm, __shfl_xor(vm, o));
        if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = vm;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = red[0];
            for (int k = 1; k < BNODES / 64; ++k) m = nmax(m, red[k]);
            a.partial[it] = m;
        }
        __syncthreads();
    }
}

// second half: one thread per instance folds its node-block maxima in order
// and retires the instance (converged or diverged); first/stride count threads
__device__ inline void bp_check_fold(const BatchArgs& a, int s, int first, int stride)
{
    for (int ii = first; ii < a.ninst; ii += stride) {
        BState& S = a.st[ii];
        if (S.status != B_RUNNING || (S.steps + s) % a.check_every != 0) continue;
        const BInst& I = a.inst[ii];
        double U = 0.0;
        for (int k = 0; k < I.nblk; ++k) U = nmax(U, a.partial[I.blk0 + k]);
        S.U_prev = S.U;
        S.U = U;
        if (!(U == U) || U - U != 0.0 || U > 0.5773502691896258) S.status = B_DIVERGED;
        else if (S.steps + s > 0 && fabs(U - S.U_prev) < a.tol) S.status = B_CONVERGED;
        if (S.status != B_RUNNING) S.stop = s;
    }
}

// collision of every running instance
template <int BNODES>
__device__ void bp_collide(const BatchArgs& a, int s, int first, int stride)
{
    for (int it = first; it < a.nblk_total; it += stride) {
        const int ii = a.blk_inst[it];
        if (a.st[ii].status != B_RUNNING) continue;
        const BInst& I = a.inst[ii];
        const int cur = (int)((a.st[ii].steps + s) & 1);
        const double* Sc = I.S[cur];
        double* Sn = I.S[1 - cur];
        const long long n = (long long)(it - I.blk0) * BNODES + threadIdx.x;
        if (n < I.g.N) {
            int x, y, z;
            coords(n, I.g, x, y, z);
            double f[9], r, jx, jy, Fx, Fy, Fz, out[9];
            b_moments(I, Sc, n, x, y, f, r, jx, jy);
            b_force_any(I, n, x, y, r, Fx, Fy, Fz);
            collide<0>(f, r, jx, jy, 0.0, Fx, Fy, Fz, I.rx, out);
#pragma unroll
            for (int i = 0; i < 9; ++i) Sn[(long long)i * I.g.ps + n] = out[i];
        }
    }
}

// Advance the step counters after the launch's last step: running instances
// took every step, the ones that retired during the launch stopped at loop
// step S.stop.  Then count the launch: the host compares this count with the
// launches it made, so a launch that did not run to here (or at all) shows as
// a missing count.  first/stride count threads.
__device__ inline void bp_finish(const BatchArgs& a, int first, int stride)
{
    for (int ii = first; ii < a.ninst; ii += stride) {
        BState& S = a.st[ii];
        if (S.status == B_RUNNING) S.steps += a.nsteps;
        else if (S.stop >= 0) S.steps += S.stop;
        S.stop = -1;
    }
    if (first == 0) *a.launches += 1u;
}

__device__ __forceinline__ void bar(cooperative_groups::grid_group& gg) { gg.sync(); }

// The persistent form: one cooperative launch runs a.nsteps steps, every
// workgroup running every phase, with grid barriers between the phases.
template <int BNODES>
__global__ void __launch_bounds__(BNODES) k_batch(BatchArgs a)
{
    namespace cg = cooperative_groups;
    cg::grid_group gg = cg::this_grid();
    // the grid barriers below exist only in a cooperative launch: any other
    // launch (a graph replay that lost the attribute) reports itself and
    // returns before the first barrier, with the state untouched
    if (!gg.is_valid()) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *a.not_cooperative = 1;
        return;
    }
    __shared__ double red[BNODES / 64];
    const int waves = BNODES / 64, wv = threadIdx.x / 64;
    for (int s = 0; s < a.nsteps; ++s) {
        bp_density<BNODES>(a, s, blockIdx.x, gridDim.x);
        bar(gg);
        // the chemical potential of the explicit schemes shares its phase
        // with the first line solves, which it does not touch
        if (a.has_compact) bp_lines<BNODES>(a, 0, blockIdx.x * waves + wv, gridDim.x * waves);
        bp_mu<BNODES>(a, blockIdx.x, gridDim.x);
        bar(gg);
        if (a.has_compact) {
            bp_lines<BNODES>(a, 1, blockIdx.x * waves + wv, gridDim.x * waves);
            bar(gg);
        }
        // convergence check on the current state (every check_every steps)
        if (bp_due<BNODES>(a, s)) {
            bp_check_partials<BNODES>(a, s, blockIdx.x, gridDim.x, red);
            bar(gg);
            bp_check_fold(a, s, blockIdx.x * BNODES + threadIdx.x, gridDim.x * BNODES);
            bar(gg);
        }
        bp_collide<BNODES>(a, s, blockIdx.x, gridDim.x);
        bar(gg);
    }
    bp_finish(a, blockIdx.x * BNODES + threadIdx.x, gridDim.x * BNODES);
}

// The phase form: the same phases as separate launches (ordinary kernels, the
// kernel boundary in place of the grid barrier), issued by the host for each
// loop step; the host issues the check kernels on the loop steps where some
// instance is due.  Every kernel strides, so any grid is correct.
template <int BNODES>
__global__ void __launch_bounds__(BNODES) k_bp_density(BatchArgs a, int s)
{
    bp_density<BNODES>(a, s, blockIdx.x, gridDim.x);
}

template <int BNODES>
__global__ void __launch_bounds__(BNODES) k_bp_mu(BatchArgs a)
{
    constexpr int waves = BNODES / 64;
    if (a.has_compact) bp_lines<BNODES>(a, 0, blockIdx.x * waves + (int)threadIdx.x / 64, gridDim.x * waves);
    bp_mu<BNODES>(a, blockIdx.x, gridDim.x);
}

template <int BNODES>
__global__ void __launch_bounds__(BNODES) k_bp_lines1(BatchArgs a)
{
    constexpr int waves = BNODES / 64;
    bp_lines<BNODES>(a, 1, blockIdx.x * waves + (int)threadIdx.x / 64, gridDim.x * waves);
}

template <int BNODES>
__global__ void __launch_bounds__(BNODES) k_bp_check(BatchArgs a, int s)
{
    __shared__ double red[BNODES / 64];
    bp_check_partials<BNODES>(a, s, blockIdx.x, gridDim.x, red);
}

template <int BNODES>
__global__ void __launch_bounds__(BNODES) k_bp_fold(BatchArgs a, int s)
{
    bp_check_fold(a, s, blockIdx.x * BNODES + threadIdx.x, gridDim.x * BNODES);
}

template <int BNODES>
__global__ void __launch_bounds__(BNODES) k_bp_collide(BatchArgs a, int s)
{
    bp_collide<BNODES>(a, s, blockIdx.x, gridDim.x);
}

template <int BNODES>
__global__ void __launch_bounds__(BNODES) k_bp_finish(BatchArgs a)
{
    bp_finish(a, blockIdx.x * BNODES + threadIdx.x, gridDim.x * BNODES);
}

}  // namespace lbm
