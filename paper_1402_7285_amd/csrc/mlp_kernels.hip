// Learned RHS-cost predictor for the work-queue scheduler (gfx950).
//
// * k_features: 16 local-environment features of each RHS orbital j, read
//   from the plan's order-N cluster map and the H / S blocks (one thread per
//   RHS).
// * A 16 -> 64 -> 64 -> 1 ReLU network in FP32.  One wave (64 lanes) handles
//   one sample at a time and lane j is hidden unit j of both layers, so a
//   layer is 64 independent dot products; hidden values pass between lanes
//   by wave shuffles and the weights sit in LDS.
// * Training: each wave accumulates the gradient of its share of the batch
//   in registers and writes it as one partial; a second kernel sums the
//   partials in a fixed order in FP64 (bitwise reproducible) and applies
//   the Adam update.
//
// Parameter layout (5313 floats): W1[64][16], b1[64], W2[64][64], b2[64],
// W3[64], b3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_params.hpp"
#include "scocg_params.hpp"

namespace scocg {

namespace mlp {

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void load_weights(const float* __restrict__ w, float* sw) {
    for (int t = threadIdx.x; t < NPARAM; t += blockDim.x) sw[t] = w[t];
    __syncthreads();
}

// Forward pass of one sample on one wave (lane j = hidden unit j); returns y
// on every lane and this lane's h1 and h2.  Hidden values move between lanes
// by wave shuffles.
__device__ __forceinline__ float forward_one(const float* sw, const float* __restrict__ xin, int lane,
                                             float* h1j, float* h2j) {
    float a = sw[OFF_B1 + lane];
#pragma unroll
    for (int i = 0; i < NIN; ++i) a += sw[OFF_W1 + lane * NIN + i] * xin[i];
    const float h1 = a > 0.f ? a : 0.f;
    float b = sw[OFF_B2 + lane];
#pragma unroll 8
    for (int k = 0; k < NH; ++k) b += sw[OFF_W2 + lane * NH + k] * __shfl(h1, k, 64);
    const float h2 = b > 0.f ? b : 0.f;
    *h1j = h1;
    *h2j = h2;
    return wsum(sw[OFF_W3 + lane] * h2) + sw[OFF_B3];
}

}  // namespace mlp

using namespace mlp;

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ w, const float* __restrict__ x,
                                                     int64_t n, float* __restrict__ y) {
    extern __shared__ float smem_f[];
    float* sw = smem_f;                              // NPARAM
    load_weights(w, sw);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t s = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv; s < n; s += nw) {
        float h1, h2;
        const float out = forward_one(sw, x + s * NIN, lane, &h1, &h2);
        if (lane == 0) y[s] = out;
    }
}

// Per-wave partial gradients of L = sum_s (y_s - t_s)^2 / n over the samples
// idx[0..m) (all samples 0..m if idx is null).
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ w, const float* __restrict__ x,
                                                  const float* __restrict__ t, const int32_t* __restrict__ idx,
                                                  int64_t m, float* __restrict__ partial,
                                                  float* __restrict__ loss_part) {
    extern __shared__ float smem_f[];
    float* sw = smem_f;
    load_weights(w, sw);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    float gW1[NIN], gW2[NH];
#pragma unroll
    for (int i = 0; i < NIN; ++i) gW1[i] = 0.f;
#pragma unroll
    for (int k = 0; k < NH; ++k) gW2[k] = 0.f;
    float gb1 = 0.f, gb2 = 0.f, gW3 = 0.f, gb3 = 0.f, lsum = 0.f;
    const float scale = 2.f / (float)m;
    for (int64_t q = gw; q < m; q += nw) {
        const int64_t s = idx ? (int64_t)idx[q] : q;
        const float* xs = x + s * NIN;
        float h1, h2;
        const float y = forward_one(sw, xs, lane, &h1, &h2);
        const float e = y - t[s];
        lsum += e * e;
        const float dy = scale * e;
        gW3 += dy * h2;
        gb3 += dy;
        const float dh2 = h2 > 0.f ? dy * sw[OFF_W3 + lane] : 0.f;
        gb2 += dh2;
#pragma unroll
        for (int k = 0; k < NH; ++k) gW2[k] += dh2 * __shfl(h1, k, 64);
        float g1 = 0.f;
#pragma unroll 8
        for (int j = 0; j < NH; ++j) g1 += sw[OFF_W2 + j * NH + lane] * __shfl(dh2, j, 64);
        const float dh1 = h1 > 0.f ? g1 : 0.f;
        gb1 += dh1;
#pragma unroll
        for (int i = 0; i < NIN; ++i) gW1[i] += dh1 * xs[i];
    }
    float* P = partial + gw * NPARAM;
#pragma unroll
    for (int i = 0; i < NIN; ++i) P[OFF_W1 + lane * NIN + i] = gW1[i];
    P[OFF_B1 + lane] = gb1;
#pragma unroll
    for (int k = 0; k < NH; ++k) P[OFF_W2 + lane * NH + k] = gW2[k];
    P[OFF_B2 + lane] = gb2;
    P[OFF_W3 + lane] = gW3;
    if (lane == 0) {
        P[OFF_B3] = gb3;
        loss_part[gw] = lsum;
    }
}

// g = sum over partials (FP64, fixed order); optional copy to grad; Adam step
// when lr > 0; loss = sum(loss_part) / m.
__global__ void k_mlp_adam(float* __restrict__ w, float* __restrict__ am, float* __restrict__ av,
                           const float* __restrict__ partial, const float* __restrict__ loss_part, int64_t nparts,
                           int64_t m, float lr, int32_t step, float* __restrict__ grad, float* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NPARAM) {
        double g = 0.0;
        for (int64_t q = 0; q < nparts; ++q) g += (double)partial[q * NPARAM + p];
        const float gf = (float)g;
        if (grad) grad[p] = gf;
        if (lr > 0.f) {
            const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
            const float mm = b1 * am[p] + (1.f - b1) * gf;
            const float vv = b2 * av[p] + (1.f - b2) * gf * gf;
            am[p] = mm;
            av[p] = vv;
            const float mh = mm / (1.f - powf(b1, (float)step));
            const float vh = vv / (1.f - powf(b2, (float)step));
            w[p] -= lr * mh / (sqrtf(vh) + eps);
        }
    }
    if (p == 0 && loss) {
        double l = 0.0;
        for (int64_t q = 0; q < nparts; ++q) l += (double)loss_part[q];
        *loss = (float)(l / (double)m);
    }
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------
__device__ __forceinline__ double blk_fro(const double* b, int bd) {
    double s = 0.0;
    for (int t = 0; t < bd * bd; ++t) s += b[t] * b[t];
    return sqrt(s);
}

__global__ void k_features(const KParams P, int bd, int has_S, float* __restrict__ feats) {
    const int rj = blockIdx.x * blockDim.x + threadIdx.x;
    if (rj >= P.nrhs) return;
    const RhsInfo ri = P.rhs[rj];
    const SysInfo si = P.sys[ri.sys];
    const int64_t* rowptr = P.rowptr_l + si.row_base;
    const int32_t* ecol = P.ecol + si.ent_base;
    const int32_t* egid = P.egid + si.ent_base;
    const double* H = P.Hv64;
    const double* S = P.Sv64;
    const int n = si.nrows;
    const int c = ri.b_local / bd, o = ri.b_local - c * bd;
    const int64_t e0 = rowptr[c], e1 = rowptr[c + 1];
    float f[NIN];
    f[0] = (float)n;
    f[1] = (float)(rowptr[n] - rowptr[0]) / (float)n;
    f[2] = (float)(e1 - e0 - 1);
    double second = 0.0;
    double hsum = 0.0, hmax = 0.0, hsq = 0.0, ssum = 0.0, gersh = 0.0;
    int nn = 0;
    double hjj = 0.0, fro_on = 0.0, glo = 0.0, ghi = 0.0;
    for (int64_t e = e0; e < e1; ++e) {
        const int b = ecol[e];
        const double* hb = H + (int64_t)egid[e] * bd * bd;
        // row o of this block contributes to the Gershgorin radius of row j
        for (int cc = 0; cc < bd; ++cc)
            if (!(b == c && cc == o)) gersh += fabs(hb[o * bd + cc]);
        if (b == c) {
            hjj = hb[o * bd + o];
            fro_on = blk_fro(hb, bd);
            glo = 1e300;
            ghi = -1e300;
            for (int r = 0; r < bd; ++r) {
                double rad = 0.0;
                for (int cc = 0; cc < bd; ++cc)
                    if (cc != r) rad += fabs(hb[r * bd + cc]);
                glo = fmin(glo, hb[r * bd + r] - rad);
                ghi = fmax(ghi, hb[r * bd + r] + rad);
            }
        } else {
            const double fr = blk_fro(hb, bd);
            hsum += fr;
            hsq += fr * fr;
            hmax = fmax(hmax, fr);
            if (has_S) ssum += blk_fro(S + (int64_t)egid[e] * bd * bd, bd);
            ++nn;
            second += (double)(rowptr[b + 1] - rowptr[b]);
        }
    }
    f[3] = (float)second;
    f[4] = o == 0 ? 1.f : 0.f;
    f[5] = (o >= 1 && o <= 3) ? 1.f : 0.f;
    f[6] = o >= 4 ? 1.f : 0.f;
    f[7] = (float)hjj;
    f[8] = (float)fro_on;
    f[9] = (float)glo;
    f[10] = (float)ghi;
    const double mean = nn ? hsum / nn : 0.0;
    f[11] = (float)mean;
    f[12] = (float)hmax;
    f[13] = (float)(nn ? sqrt(fmax(0.0, hsq / nn - mean * mean)) : 0.0);
    f[14] = (float)gersh;
    f[15] = (float)(nn ? ssum / nn : 0.0);
#pragma unroll
    for (int i = 0; i < NIN; ++i) feats[(int64_t)rj * NIN + i] = f[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static size_t mlp_lds_bytes() { return sizeof(float) * NPARAM_PAD; }

hipError_t launch_mlp_forward(const float* w, const float* x, int64_t n, float* y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 3) / 4, 1024);
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), mlp_lds_bytes(), st, w, x, n, y);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* w, const float* x, const float* t, const int32_t* idx, int64_t m,
                           float* partial, float* loss_part, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblocks), dim3(256), mlp_lds_bytes(), st, w, x, t, idx, m, partial,
                       loss_part);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* w, float* am, float* av, const float* partial, const float* loss_part,
                           int64_t nparts, int64_t m, float lr, int32_t step, float* grad, float* loss,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, w, am, av, partial, loss_part,
                       nparts, m, lr, step, grad, loss);
    return hipGetLastError();
}

hipError_t launch_features(const KParams& P, int bd, int has_S, float* feats, hipStream_t st) {
    if (P.nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3((P.nrhs + 127) / 128), dim3(128), 0, st, P, bd, has_S, feats);
    return hipGetLastError();
}

}  // namespace scocg
