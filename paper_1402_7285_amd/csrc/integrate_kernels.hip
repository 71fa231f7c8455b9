// Energy integration of the Green's-function output (gfx950).
//
// After a solve, the output holds G_ij(z_k) for every RHS j, shift k and
// requested row i, laid out [rhs][shift][row].  Integrating over the real
// parts E_k of the shifts gives what G is used for (the density of states
// and the density matrix of the electronic structure, Sec. 2-3):
//
//   rho_ij      = -(1/pi) sum_k w_k f(E_k) Im G_ij(z_k)
//   ldos_j(E_k) = -(1/pi) Im G_jj(z_k)
//
// with caller-supplied quadrature weights w_k and the Fermi function
// f(E) = 1/(1 + exp((E - mu)/kT)), computed as (1 - tanh((E - mu)/(2 kT)))/2
// (no overflow), a step with 1/2 at E = mu for kT = 0.  One workgroup per
// RHS (grid-stride): w_k f(E_k) is formed once in LDS, then each thread sums
// over k for its rows in order k = 0, 1, ... (reads of one k are contiguous
// over rows).  The kernel reads the output once: it is bound by HBM.
#include <hip/hip_runtime.h>
#include <math.h>

#include "scocg_params.hpp"

namespace scocg {

__global__ __launch_bounds__(256) void k_integrate(const double* __restrict__ G, const double* __restrict__ z,
                                                   const double* __restrict__ w, const RhsInfo* __restrict__ rhs,
                                                   const int64_t* __restrict__ out_off,
                                                   const int32_t* __restrict__ out_local, int nrhs, int K,
                                                   double mu, double kT, double* __restrict__ rho,
                                                   double* __restrict__ ldos) {
    extern __shared__ double wf[];       // K weights times occupations
    __shared__ int diag;
    constexpr double inv_pi = 0.318309886183790671537767526745;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const double E = z[2 * k];
        double f;
        if (kT > 0.0) f = 0.5 * (1.0 - tanh(0.5 * (E - mu) / kT));
        else f = E < mu ? 1.0 : (E > mu ? 0.0 : 0.5);
        wf[k] = w[k] * f;
    }
    for (int rj = blockIdx.x; rj < nrhs; rj += gridDim.x) {
        const RhsInfo ri = rhs[rj];
        const int n = ri.nout;
        const int64_t row0 = out_off[rj];
        const double* g = G + 2 * row0 * (int64_t)K;      // [K][n] complex
        if (threadIdx.x == 0) diag = ri.full_x ? ri.b_local : -1;
        __syncthreads();
        if (!ri.full_x)
            for (int o = threadIdx.x; o < n; o += blockDim.x)
                if (out_local[ri.out_base + o] == ri.b_local) diag = o;   // at most one row matches
        __syncthreads();
        for (int o = threadIdx.x; o < n; o += blockDim.x) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc += wf[k] * g[2 * ((int64_t)k * n + o) + 1];
            rho[row0 + o] = -acc * inv_pi;
        }
        if (ldos) {
            const int d = diag;
            for (int k = threadIdx.x; k < K; k += blockDim.x)
                ldos[(int64_t)rj * K + k] = d >= 0 ? -g[2 * ((int64_t)k * n + d) + 1] * inv_pi : NAN;
        }
        __syncthreads();
    }
}

hipError_t launch_integrate(const double* G, const double* z, const double* w, const RhsInfo* rhs,
                            const int64_t* out_off, const int32_t* out_local, int nrhs, int K, double mu, double kT,
                            double* rho, double* ldos, hipStream_t st) {
    if (nrhs <= 0) return hipSuccess;
    const int blocks = nrhs < 4096 ? nrhs : 4096;
    hipLaunchKernelGGL(k_integrate, dim3(blocks), dim3(256), sizeof(double) * (size_t)K, st, G, z, w, rhs, out_off,
                       out_local, nrhs, K, mu, kT, rho, ldos);
    return hipGetLastError();
}

// Integrated crystal-orbital Hamilton population of each output pair:
// cohp[o] = H_{row(o), j} rho[o], with H_{row(o), j} gathered per output row
// on the host when the plan is built.  Elementwise and bound by HBM.
__global__ __launch_bounds__(256) void k_cohp(const double* __restrict__ h, const double* __restrict__ rho,
                                              double* __restrict__ cohp, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        cohp[t] = h[t] * rho[t];
}

hipError_t launch_cohp(const double* h, const double* rho, double* cohp, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 255) / 256;
    const int blocks = (int)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(k_cohp, dim3(blocks), dim3(256), 0, st, h, rho, cohp, n);
    return hipGetLastError();
}

}  // namespace scocg
