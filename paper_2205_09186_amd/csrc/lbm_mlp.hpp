// lbm_mlp.hpp -- FP32 kernels of the learned initialiser: a 4 -> 64 -> 64 ->
// 64 -> 1 network with SiLU activations that maps (Tr, k, scheme, signed
// distance to the interface) to the normalised equilibrium density
// phi = (rho - rho_g) / (rho_l - rho_g).  Forward, mean-squared-error gradient,
// backpropagation with a deterministic (fixed-order) batch reduction, Adam,
// and whole-field inference that writes an initial density for the step.
//
// Flat parameter layout (8705 floats): W1 (64 x 4, row = output), b1, W2
// (64 x 64), b2, W3 (64 x 64), b3, W4 (1 x 64), b4.
#pragma once

#include <hip/hip_runtime.h>
#include "lbm_kernels.hpp"

namespace lbm {

constexpr int MH = 64, MI = 4;
constexpr int OW1 = 0, OB1 = OW1 + MH * MI, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH,
              OB3 = OW3 + MH * MH, OW4 = OB3 + MH, OB4 = OW4 + MH, MP = OB4 + 1;   // 8705
constexpr int MACT = 3 * MH;   // stored pre-activations per sample
constexpr int MB = 64;         // samples per workgroup
constexpr int LP = MB + 1;     // padded LDS row (bank spread)

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z)
{
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

struct MlpNorm {   // feature scaling: (v - shift) * scale; distance / dscale
    float tr0, trs, k0, ks, s0, ss, dscale;
};

// One sample through the network; pre-activations to zs (may be null).
// hb is this thread's column of a [MH][LP] LDS buffer.
__device__ __forceinline__ float mlp_eval(const float* __restrict__ w, const float (&x)[MI], float* hb, int tid,
                                          float* zs)
{
    float h[MH];
    for (int o = 0; o < MH; ++o) {
        float z = w[OB1 + o];
#pragma unroll
        for (int i = 0; i < MI; ++i) z += w[OW1 + o * MI + i] * x[i];
        if (zs) zs[o] = z;
        hb[o * LP + tid] = silu_f(z);
    }
#pragma unroll
    for (int i = 0; i < MH; ++i) h[i] = hb[i * LP + tid];
    for (int layer = 0; layer < 2; ++layer) {
        const int ow = layer == 0 ? OW2 : OW3, ob = layer == 0 ? OB2 : OB3;
        for (int o = 0; o < MH; ++o) {
            float z = w[ob + o];
#pragma unroll
            for (int i = 0; i < MH; ++i) z += w[ow + o * MH + i] * h[i];
            if (zs) zs[(layer + 1) * MH + o] = z;
            hb[o * LP + tid] = silu_f(z);
        }
#pragma unroll
        for (int i = 0; i < MH; ++i) h[i] = hb[i * LP + tid];
    }
    float y = w[OB4];
#pragma unroll
    for (int i = 0; i < MH; ++i) y += w[OW4 + i] * h[i];
    return y;
}

__global__ void __launch_bounds__(MB) k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ X, int B,
                                                float* __restrict__ Y, float* __restrict__ acts)
{
    __shared__ float w[MP];
    __shared__ float hb[MH * LP];
    for (int j = threadIdx.x; j < MP; j += MB) w[j] = P[j];
    __syncthreads();
    const int s = blockIdx.x * MB + threadIdx.x;
    float x[MI];
#pragma unroll
    for (int i = 0; i < MI; ++i) x[i] = s < B ? X[(long long)s * MI + i] : 0.0f;
    float* zs = (acts && s < B) ? acts + (long long)s * MACT : nullptr;
    const float y = mlp_eval(w, x, hb, threadIdx.x, zs);
    if (s < B) Y[s] = y;
}

// dY = 2 (y - t) / B; per-workgroup partial sums of (y - t)^2.
__global__ void __launch_bounds__(MB) k_mlp_loss(const float* __restrict__ Y, const float* __restrict__ T, int B,
                                                 float* __restrict__ dY, float* __restrict__ lpart)
{
    __shared__ float r[MB];
    const int s = blockIdx.x * MB + threadIdx.x;
    float e = 0.0f;
    if (s < B) {
        e = Y[s] - T[s];
        dY[s] = 2.0f * e / (float)B;
    }
    r[threadIdx.x] = e * e;
    __syncthreads();
    if (threadIdx.x == 0) {
        float a = 0.0f;
        for (int k = 0; k < MB; ++k) a += r[k];
        lpart[blockIdx.x] = a;
    }
}

// Backpropagation of one workgroup of samples; writes that workgroup's
// parameter-gradient partial sums (samples summed in index order).
__global__ void __launch_bounds__(MB) k_mlp_bwd(const float* __restrict__ P, const float* __restrict__ X,
                                                const float* __restrict__ acts, const float* __restrict__ dY, int B,
                                                float* __restrict__ gpart)
{
    __shared__ float w[MP];
    __shared__ float d[3][MH * LP];    // deltas of layers 1..3
    __shared__ float hh[3][MH * LP];   // activations of layers 1..3
    __shared__ float xs[MI * LP];
    __shared__ float dys[MB];
    for (int j = threadIdx.x; j < MP; j += MB) w[j] = P[j];
    const int t = threadIdx.x;
    const int s = blockIdx.x * MB + t;
    const bool valid = s < B;
    const float dy = valid ? dY[s] : 0.0f;
    dys[t] = dy;
#pragma unroll
    for (int i = 0; i < MI; ++i) xs[i * LP + t] = valid ? X[(long long)s * MI + i] : 0.0f;
    const float* z = valid ? acts + (long long)s * MACT : nullptr;
    for (int l = 0; l < 3; ++l)
        for (int i = 0; i < MH; ++i) hh[l][i * LP + t] = valid ? silu_f(z[l * MH + i]) : 0.0f;
    __syncthreads();
    // layer 3 delta: W4^T dy * silu'(z3)
    for (int i = 0; i < MH; ++i) d[2][i * LP + t] = valid ? w[OW4 + i] * dy * dsilu_f(z[2 * MH + i]) : 0.0f;
    // layers 2 and 1: delta_l = (W_{l+1}^T delta_{l+1}) * silu'(z_l)
    for (int l = 1; l >= 0; --l) {
        const int ow = l == 1 ? OW3 : OW2;
        for (int i = 0; i < MH; ++i) {
            float a = 0.0f;
            for (int o = 0; o < MH; ++o) a += w[ow + o * MH + i] * d[l + 1][o * LP + t];
            d[l][i * LP + t] = valid ? a * dsilu_f(z[l * MH + i]) : 0.0f;
        }
    }
    __syncthreads();
    float* g = gpart + (long long)blockIdx.x * MP;
    for (int j = t; j < MP; j += MB) {
        float a = 0.0f;
        if (j < OB1) {                       // W1
            const int o = j / MI, i = j % MI;
            for (int k = 0; k < MB; ++k) a += d[0][o * LP + k] * xs[i * LP + k];
        } else if (j < OW2) {                // b1
            const int o = j - OB1;
            for (int k = 0; k < MB; ++k) a += d[0][o * LP + k];
        } else if (j < OB2) {                // W2
            const int o = (j - OW2) / MH, i = (j - OW2) % MH;
            for (int k = 0; k < MB; ++k) a += d[1][o * LP + k] * hh[0][i * LP + k];
        } else if (j < OW3) {                // b2
            const int o = j - OB2;
            for (int k = 0; k < MB; ++k) a += d[1][o * LP + k];
        } else if (j < OB3) {                // W3
            const int o = (j - OW3) / MH, i = (j - OW3) % MH;
            for (int k = 0; k < MB; ++k) a += d[2][o * LP + k] * hh[1][i * LP + k];
        } else if (j < OW4) {                // b3
            const int o = j - OB3;
            for (int k = 0; k < MB; ++k) a += d[2][o * LP + k];
        } else if (j < OB4) {                // W4
            const int i = j - OW4;
            for (int k = 0; k < MB; ++k) a += dys[k] * hh[2][i * LP + k];
        } else {                             // b4
            for (int k = 0; k < MB; ++k) a += dys[k];
        }
        g[j] = a;
    }
}

// Sum of the per-workgroup partials, workgroups in order.
__global__ void __launch_bounds__(256) k_mlp_gsum(const float* __restrict__ gpart, int nb, float* __restrict__ G)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= MP) return;
    float a = 0.0f;
    for (int b = 0; b < nb; ++b) a += gpart[(long long)b * MP + j];
    G[j] = a;
}

__global__ void __launch_bounds__(256) k_adam(float* __restrict__ P, const float* __restrict__ G,
                                              float* __restrict__ M, float* __restrict__ V, float lr, float b1,
                                              float b2, float eps, float c1, float c2)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= MP) return;
    const float g = G[j];
    const float m = b1 * M[j] + (1.0f - b1) * g;
    const float v = b2 * V[j] + (1.0f - b2) * g * g;
    M[j] = m;
    V[j] = v;
    P[j] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Initial density of every node from the network: signed distance to a
// sphere (circle) of radius R around (cx, cy, cz); phi clamped to [0, 1].
__global__ void __launch_bounds__(MB) k_mlp_field(const float* __restrict__ P, MlpNorm nm, Grid g, double cx,
                                                  double cy, double cz, double R, float ftr, float fk, float fs,
                                                  double rho_g, double rho_l, double* __restrict__ out)
{
    __shared__ float w[MP];
    __shared__ float hb[MH * LP];
    for (int j = threadIdx.x; j < MP; j += MB) w[j] = P[j];
    __syncthreads();
    const long long n = (long long)blockIdx.x * MB + threadIdx.x;
    int x = 0, y = 0, z = 0;
    if (n < g.N) coords(n, g, x, y, z);
    const double dx = x - cx, dy = y - cy, dz = z - cz;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    float in[MI] = { ftr, fk, fs, (float)((r - R) / nm.dscale) };
    float phi = mlp_eval(w, in, hb, threadIdx.x, nullptr);
    phi = fminf(fmaxf(phi, 0.0f), 1.0f);
    if (n < g.N) out[n] = rho_g + (double)phi * (rho_l - rho_g);
}

// Deterministic sum: per-workgroup partials (fixed tree), reduced by
// k_reduce_final.
__global__ void __launch_bounds__(256) k_sum_partials(const double* __restrict__ x, long long N,
                                                      double* __restrict__ partial)
{
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    double mx = 0.0, sm = n < N ? x[n] : 0.0;
    block_reduce<256>(mx, sm);
    if (threadIdx.x == 0) { partial[2 * blockIdx.x] = 0.0; partial[2 * blockIdx.x + 1] = sm; }
}

// Interface mass: the weight w = phi (1 - phi) of a node, phi = (rho -
// rho_g)/(rho_l - rho_g) clamped to [0, 1], is zero on both plateaus.
__device__ __forceinline__ double iface_w(double r, double rg, double rl)
{
    const double phi = fmin(fmax((r - rg) / (rl - rg), 0.0), 1.0);
    return phi * (1.0 - phi);
}

// Two sums over a workgroup in a fixed order (wavefront tree, then waves in
// order); thread 0 holds the result.
template <int BS>
__device__ __forceinline__ void block_sum2(double& a, double& b)
{
    __shared__ double sa[BS / 64], sb[BS / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
    if (ln == 0) { sa[wv] = a; sb[wv] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = sa[0]; b = sb[0];
        for (int k = 1; k < BS / 64; ++k) { a += sa[k]; b += sb[k]; }
    }
}

__global__ void __launch_bounds__(256) k_mass_partials(const double* __restrict__ rho, long long N, double rg,
                                                       double rl, double* __restrict__ partial)
{
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    double m = 0.0, w = 0.0;
    if (n < N) { m = rho[n]; w = iface_w(m, rg, rl); }
    block_sum2<256>(m, w);
    if (threadIdx.x == 0) { partial[2 * blockIdx.x] = m; partial[2 * blockIdx.x + 1] = w; }
}

__global__ void __launch_bounds__(1024) k_mass_final(const double* __restrict__ partial, long long nb,
                                                     double* __restrict__ out)
{
    double m = 0.0, w = 0.0;
    for (long long k = threadIdx.x; k < nb; k += 1024) {
        m += partial[2 * k];
        w += partial[2 * k + 1];
    }
    block_sum2<1024>(m, w);
    if (threadIdx.x == 0) { out[0] = m; out[1] = w; }
}

// rho += (target - M) w / W on every node (M, W in tot); nothing where W = 0.
__global__ void __launch_bounds__(256) k_mass_apply(double* __restrict__ rho, long long N, double rg, double rl,
                                                    const double* __restrict__ tot, double target)
{
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    const double W = tot[1];
    if (n >= N || !(W > 0.0)) return;
    const double r = rho[n];
    rho[n] = r + (target - tot[0]) * (iface_w(r, rg, rl) / W);
}

}  // namespace lbm
