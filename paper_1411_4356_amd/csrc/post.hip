// Post-processing of a steady-state solution and the parameter derivatives
// used by adjoint gradients.
//
// x is vec(rho) in the ordering of the matrix (permuted by RCM or natural):
// the natural position p of an entry is stored at iperm[p].  The diagonal of
// rho sits at natural positions k (N + 1).  Observables (Sec. IV):
// <a^dag a> = sum_k i_k rho_kk, <b^dag b> = sum_k j_k rho_kk,
// F = (<(b^dag b)^2> - <b^dag b>^2) / <b^dag b>, with rho = x / Tr x.
//
// Gradients: for an objective f = Re o^T x of the solution of the constrained
// system, df/dtheta = -Re lambda^H P0 (dL/dtheta) x with A^H lambda = conj(o);
// P0 removes row 0 (the trace row, whose derivative multiplies Tr x - 1 = 0).
// dL/dtheta is the stencil evaluated at a unit parameter set.
#include <vector>

#include "common.hpp"
#include "cplx.hpp"
#include "kernels.hpp"
#include "post.hpp"
#include "stencil.hpp"

namespace omss {

constexpr int PT = 256;

__device__ inline double psum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// per item: out[b*8 + 0..7] = tr.re, tr.im, Sa.re, Sa.im, Sb.re, Sb.im, Sb2.re, Sb2.im
__global__ __launch_bounds__(PT) void diag_sums_kernel(const double2* __restrict__ x, int64_t n, int N, int nm,
                                                      const int32_t* __restrict__ iperm, double* __restrict__ out) {
    const int b = blockIdx.x;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < N; k += PT) {
        const int64_t p = (int64_t)k * (N + 1);
        const double2 v = x[(int64_t)b * n + (iperm ? iperm[p] : p)];
        const double i = (double)(k / nm), j = (double)(k % nm);
        acc[0] += v.x; acc[1] += v.y;
        acc[2] += i * v.x; acc[3] += i * v.y;
        acc[4] += j * v.x; acc[5] += j * v.y;
        acc[6] += j * j * v.x; acc[7] += j * j * v.y;
    }
    __shared__ double red[PT / 64][8];
    for (int q = 0; q < 8; ++q) {
        const double s = psum(acc[q]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double s = 0;
        for (int w = 0; w < PT / 64; ++w) s += red[w][threadIdx.x];
        out[b * 8 + threadIdx.x] = s;
    }
}

// obs[b*3 + (0,1,2)] = n_a, n_b, F from the diagonal sums
__global__ void observables_kernel(const double* __restrict__ sums, int batch, double* __restrict__ obs,
                                   double* __restrict__ trace_out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const double* s = sums + b * 8;
    const double tr = s[0], ti = s[1];
    const double den = tr * tr + ti * ti;
    // Re(S / tr)
    auto re_div = [&](double a, double c) { return (a * tr + c * ti) / den; };
    const double na = re_div(s[2], s[3]);
    const double nb = re_div(s[4], s[5]);
    const double nb2 = re_div(s[6], s[7]);
    obs[b * 3 + 0] = na;
    obs[b * 3 + 1] = nb;
    obs[b * 3 + 2] = nb != 0.0 ? (nb2 - nb * nb) / nb : 0.0;
    if (trace_out) { trace_out[2 * b] = tr; trace_out[2 * b + 1] = ti; }
}

// rho[b][p] = x[b][iperm[p]] / tr[b], p natural (column-major rho)
__global__ __launch_bounds__(PT) void unvec_kernel(const double2* __restrict__ x, int64_t n,
                                                   const int32_t* __restrict__ iperm, const double* __restrict__ trace,
                                                   double2* __restrict__ rho) {
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * PT + threadIdx.x;
    if (p >= n) return;
    const double2 v = x[(int64_t)b * n + (iperm ? iperm[p] : p)];
    const double tr = trace[2 * b], ti = trace[2 * b + 1];
    const double den = tr * tr + ti * ti;
    rho[(int64_t)b * n + p] = make_double2((v.x * tr + v.y * ti) / den, (v.y * tr - v.x * ti) / den);
}

// partial sums of |rho - rho^H|^2 and |rho|^2 over natural positions
__global__ __launch_bounds__(PT) void herm_kernel(const double2* __restrict__ rho, int64_t n, int N,
                                                  double* __restrict__ part) {
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * PT + threadIdx.x;
    double d2 = 0, r2 = 0;
    if (p < n) {
        const int64_t l = p / N, k = p - l * N;
        const double2 a = rho[(int64_t)b * n + p];
        const double2 c = rho[(int64_t)b * n + k * N + l];
        const double dx = a.x - c.x, dy = a.y + c.y;
        d2 = dx * dx + dy * dy;
        r2 = a.x * a.x + a.y * a.y;
    }
    __shared__ double red[PT / 64][2];
    d2 = psum(d2);
    r2 = psum(r2);
    if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6][0] = d2; red[threadIdx.x >> 6][1] = r2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0;
        for (int w = 0; w < PT / 64; ++w) { s0 += red[w][0]; s1 += red[w][1]; }
        part[((int64_t)b * gridDim.x + blockIdx.x) * 2 + 0] = s0;
        part[((int64_t)b * gridDim.x + blockIdx.x) * 2 + 1] = s1;
    }
}

// g[(f*batch + b)*n + iperm[k(N+1)]] = o_f(k) (real) for f = n_a, n_b, F
__global__ __launch_bounds__(PT) void objective_kernel(int64_t n, int N, int nm, int batch,
                                                      const int32_t* __restrict__ iperm, const double* __restrict__ obs,
                                                      double2* __restrict__ g) {
    const int b = blockIdx.y;
    const int k = blockIdx.x * PT + threadIdx.x;
    if (k >= N) return;
    const int64_t p = (int64_t)k * (N + 1);
    const int64_t at = iperm ? iperm[p] : p;
    const double i = (double)(k / nm), j = (double)(k % nm);
    const double m1 = obs[b * 3 + 1], F = obs[b * 3 + 2];
    g[((int64_t)0 * batch + b) * n + at] = make_double2(i, 0.0);
    g[((int64_t)1 * batch + b) * n + at] = make_double2(j, 0.0);
    g[((int64_t)2 * batch + b) * n + at] = make_double2(j * j / m1 - (2.0 + F / m1) * j, 0.0);
}

// Per block partial sums of -Re lambda_f^H (dL/dtheta_t x) over rows p >= 1,
// part[((b * nblk + blk) * nrhs + f) * 5 + t].
__global__ __launch_bounds__(PT) void grad_kernel(Dims d, const DevParams* __restrict__ unit /*5 per item*/,
                                                  const double2* __restrict__ x, const double2* __restrict__ lam,
                                                  int nrhs, int batch, const int32_t* __restrict__ iperm,
                                                  double* __restrict__ part) {
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * PT + threadIdx.x;
    const int64_t n = d.n;
    double acc[3 * 5];
    for (int q = 0; q < 15; ++q) acc[q] = 0;
    if (p >= 1 && p < n) {
        double2 dv[5];
        for (int t = 0; t < 5; ++t) dv[t] = make_double2(0.0, 0.0);
        for (int s = 0; s < NSLOT; ++s) {
            int64_t q;
            double2 v;
            if (!stencil_entry(s, p, d, unit[b * 5 + 0], q, v)) continue;
            const double2 xv = x[(int64_t)b * n + (iperm ? iperm[q] : q)];
            for (int t = 0; t < 5; ++t) {
                stencil_entry(s, p, d, unit[b * 5 + t], q, v);
                dv[t].x += v.x * xv.x - v.y * xv.y;
                dv[t].y += v.x * xv.y + v.y * xv.x;
            }
        }
        const int64_t pp = iperm ? iperm[p] : p;
        for (int f = 0; f < nrhs; ++f) {
            const double2 l = lam[((int64_t)f * batch + b) * n + pp];
            for (int t = 0; t < 5; ++t) acc[f * 5 + t] = -(l.x * dv[t].x + l.y * dv[t].y);   // -Re conj(l) dv
        }
    }
    __shared__ double red[PT / 64][15];
    for (int q = 0; q < nrhs * 5; ++q) {
        const double s = psum(acc[q]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < nrhs * 5) {
        double s = 0;
        for (int w = 0; w < PT / 64; ++w) s += red[w][threadIdx.x];
        part[((int64_t)b * gridDim.x + blockIdx.x) * (nrhs * 5) + threadIdx.x] = s;
    }
}

om_status observables(const om_csr* A, const double2* x, double* obs_dev, double* trace_dev, hipStream_t s) {
    if (!A->has_model) { set_error("matrix carries no model description"); return OM_EINVAL; }
    DevBuf<double> sums;
    OM_TRY(sums.alloc((size_t)A->batch * 8));
    const int nm = A->params[0].nm;
    hipLaunchKernelGGL(diag_sums_kernel, dim3(A->batch), dim3(PT), 0, s, x, A->n, A->N, nm,
                       A->permuted ? A->iperm_d.p : nullptr, sums.p);
    hipLaunchKernelGGL(observables_kernel, dim3(blocks_for(A->batch, 64)), dim3(64), 0, s, sums.p, A->batch, obs_dev,
                       trace_dev);
    OM_HIP(hipGetLastError());
    OM_HIP(hipStreamSynchronize(s));
    return OM_OK;
}

om_status unvec(const om_csr* A, const double2* x, const double* trace_dev, double2* rho, double* herm_err_host,
                hipStream_t s) {
    dim3 grid(blocks_for(A->n, PT), A->batch);
    hipLaunchKernelGGL(unvec_kernel, grid, dim3(PT), 0, s, x, A->n, A->permuted ? A->iperm_d.p : nullptr, trace_dev, rho);
    OM_HIP(hipGetLastError());
    if (herm_err_host) {
        DevBuf<double> part;
        OM_TRY(part.alloc((size_t)A->batch * grid.x * 2));
        hipLaunchKernelGGL(herm_kernel, grid, dim3(PT), 0, s, rho, A->n, A->N, part.p);
        OM_HIP(hipGetLastError());
        std::vector<double> h((size_t)A->batch * grid.x * 2);
        OM_HIP(hipMemcpyAsync(h.data(), part.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        OM_HIP(hipStreamSynchronize(s));
        for (int b = 0; b < A->batch; ++b) {
            double d2 = 0, r2 = 0;
            for (unsigned t = 0; t < grid.x; ++t) { d2 += h[((size_t)b * grid.x + t) * 2]; r2 += h[((size_t)b * grid.x + t) * 2 + 1]; }
            herm_err_host[b] = r2 > 0 ? std::sqrt(d2 / r2) : 0.0;
        }
    }
    return OM_OK;
}

om_status objective_vectors(const om_csr* A, const double2* x, double2* g, hipStream_t s) {
    DevBuf<double> obs;
    OM_TRY(obs.alloc((size_t)A->batch * 3));
    OM_TRY(observables(A, x, obs.p, nullptr, s));
    OM_HIP(hipMemsetAsync(g, 0, (size_t)3 * A->batch * A->n * sizeof(double2), s));
    dim3 grid(blocks_for(A->N, PT), A->batch);
    hipLaunchKernelGGL(objective_kernel, grid, dim3(PT), 0, s, A->n, A->N, A->params[0].nm, A->batch,
                       A->permuted ? A->iperm_d.p : nullptr, obs.p, g);
    OM_HIP(hipGetLastError());
    OM_HIP(hipStreamSynchronize(s));
    return OM_OK;
}

om_status param_gradient(const om_csr* A, const double2* x, const double2* lam, int nrhs, double* grad_host,
                         hipStream_t s) {
    if (!A->has_model) { set_error("matrix carries no model description"); return OM_EINVAL; }
    if (nrhs < 1 || nrhs > 3) { set_error("nrhs must be 1..3"); return OM_EINVAL; }
    const om_params& p0 = A->params[0];
    Dims d{p0.nc, p0.nm, p0.nc * p0.nm, A->n};
    std::vector<DevParams> unit((size_t)A->batch * 5);
    for (int b = 0; b < A->batch; ++b) {
        const double nth = A->params[b].n_th;
        unit[b * 5 + 0] = DevParams{1.0, 0.0, 0.0, 0.0, 0.0, 0.0, nth};   // Delta
        unit[b * 5 + 1] = DevParams{0.0, 0.0, 1.0, 0.0, 0.0, 0.0, nth};   // g0
        unit[b * 5 + 2] = DevParams{0.0, 0.0, 0.0, 1.0, 0.0, 0.0, nth};   // E
        unit[b * 5 + 3] = DevParams{0.0, 0.0, 0.0, 0.0, 1.0, 0.0, nth};   // kappa
        unit[b * 5 + 4] = DevParams{0.0, 0.0, 0.0, 0.0, 0.0, 1.0, nth};   // Gamma_m
    }
    DevBuf<DevParams> du;
    OM_TRY(du.upload(unit.data(), unit.size(), s));
    dim3 grid(blocks_for(A->n, PT), A->batch);
    DevBuf<double> part;
    OM_TRY(part.alloc((size_t)A->batch * grid.x * nrhs * 5));
    hipLaunchKernelGGL(grad_kernel, grid, dim3(PT), 0, s, d, du.p, x, lam, nrhs, A->batch,
                       A->permuted ? A->iperm_d.p : nullptr, part.p);
    OM_HIP(hipGetLastError());
    std::vector<double> h(part.n);
    OM_HIP(hipMemcpyAsync(h.data(), part.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    OM_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < A->batch; ++b)
        for (int q = 0; q < nrhs * 5; ++q) {
            double acc = 0;
            for (unsigned t = 0; t < grid.x; ++t) acc += h[((size_t)b * grid.x + t) * nrhs * 5 + q];
            grad_host[(size_t)b * nrhs * 5 + q] = acc;
        }
    return OM_OK;
}

}  // namespace omss
