// Restarted GMRES(m) with right preconditioning, batched over the items of a
// parameter batch (Sec. IV uses restarted GMRES with an ILU preconditioner).
//
// Right preconditioning (A M^{-1} u = b, x = M^{-1} u) keeps the Arnoldi
// residual equal to the true residual; the paper writes the left form Eq. (6),
// which has the same solution.  Per Arnoldi step j and batch item:
//   z = M^{-1} v_j, w = A z,
//   classical Gram-Schmidt twice: h = V_j^H w, w -= V_j h (FP64 dot products),
//   beta = ||w||, v_{j+1} = w / beta,
//   Givens rotations of the Hessenberg column and the residual estimate, all
//   in FP64 on the device.
// At the end of a cycle, y solves the triangular system, u = V y and
// x += M^{-1} u; the FP64 true residual ||b - A x|| / ||b|| decides
// convergence.  Basis vectors are stored [k][item][n] so that v_j of every
// item is one contiguous batch vector.
//
// The core is templated on the complex type: complex128 for the plain FP64
// solve and complex64 for the inner solves of mixed-precision iterative
// refinement (GMRES-IR), whose outer residual and update stay in FP64.
#include <chrono>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "cplx.hpp"
#include "gmres.hpp"
#include "kernels.hpp"
#include "profile.hpp"

namespace omss {

constexpr int BT = 256;
constexpr int RPT = 4;
constexpr int TILE = BT * RPT;
constexpr int KMAX = 128;

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ inline double block_sum(double v) {
    __shared__ double red[BT / 64];
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BT / 64; ++w) t += red[w];
    return t;   // valid in thread 0
}

// out[b] = sum_t part[b * np + t]
__global__ __launch_bounds__(BT) void sum_partials_kernel(const double* __restrict__ part, int np, double* __restrict__ out) {
    const int b = blockIdx.x;
    double s = 0;
    for (int t = threadIdx.x; t < np; t += BT) s += part[(int64_t)b * np + t];
    s = block_sum(s);
    if (threadIdx.x == 0) out[b] = s;
}

template <typename VT>
__global__ __launch_bounds__(BT) void norm2_partial_kernel(const VT* __restrict__ x, int64_t n, double* __restrict__ part) {
    const int b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    double s = 0;
    if (i < n) {
        const double2 v = to64(x[(int64_t)b * n + i]);
        s = v.x * v.x + v.y * v.y;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[(int64_t)b * gridDim.x + blockIdx.x] = s;
}

// part[((b * ntile) + tile) * KMAX + k] = sum_{i in tile} conj(V_k[b][i]) w[b][i]
template <typename VT>
__global__ __launch_bounds__(BT) void mdot_kernel(const VT* __restrict__ V, int64_t kstride, int64_t n, int nk,
                                                  const VT* __restrict__ w, double2* __restrict__ part,
                                                  const int32_t* __restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ double2 red[BT / 64][KMAX];
    double2 wr[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int64_t i = base + (int64_t)r * BT + threadIdx.x;
        wr[r] = i < n ? to64(w[(int64_t)b * n + i]) : make_double2(0.0, 0.0);
    }
    const VT* Vb = V + (int64_t)b * n;
    for (int k = 0; k < nk; ++k) {
        double ar = 0, ai = 0;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int64_t i = base + (int64_t)r * BT + threadIdx.x;
            if (i < n) {
                const double2 v = to64(Vb[(int64_t)k * kstride + i]);
                ar += v.x * wr[r].x + v.y * wr[r].y;
                ai += v.x * wr[r].y - v.y * wr[r].x;
            }
        }
        ar = wave_sum(ar);
        ai = wave_sum(ai);
        if (lane == 0) red[wave][k] = make_double2(ar, ai);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += BT) {
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int wv = 0; wv < BT / 64; ++wv) { s.x += red[wv][k].x; s.y += red[wv][k].y; }
        part[((int64_t)b * gridDim.x + blockIdx.x) * KMAX + k] = s;
    }
}

// h[b*KMAX+k] = sum over tiles; hsum = h (first pass) or hsum += h
__global__ void mdot_finalize_kernel(const double2* __restrict__ part, int ntile, int nk, double2* __restrict__ h,
                                     double2* __restrict__ hsum, int accumulate, const int32_t* __restrict__ active) {
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    for (int k = threadIdx.x; k < nk; k += blockDim.x) {
        double2 s = make_double2(0.0, 0.0);
        for (int t = 0; t < ntile; ++t) {
            const double2 v = part[((int64_t)b * ntile + t) * KMAX + k];
            s.x += v.x;
            s.y += v.y;
        }
        h[b * KMAX + k] = s;
        if (accumulate) { hsum[b * KMAX + k].x += s.x; hsum[b * KMAX + k].y += s.y; }
        else hsum[b * KMAX + k] = s;
    }
}

// w -= sum_k V_k h_k (FP64 arithmetic); optional squared-norm partials
template <typename VT>
__global__ __launch_bounds__(BT) void update_kernel(const VT* __restrict__ V, int64_t kstride, int64_t n, int nk,
                                                    const double2* __restrict__ h, VT* __restrict__ w,
                                                    double* __restrict__ norm2, const int32_t* __restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    __shared__ double2 hs[KMAX];
    for (int k = threadIdx.x; k < nk; k += BT) hs[k] = h[b * KMAX + k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    double sq = 0;
    if (i < n) {
        double2 acc = to64(w[(int64_t)b * n + i]);
        const VT* Vb = V + (int64_t)b * n + i;
        for (int k = 0; k < nk; ++k) {
            const double2 v = to64(Vb[(int64_t)k * kstride]);
            acc.x -= v.x * hs[k].x - v.y * hs[k].y;
            acc.y -= v.x * hs[k].y + v.y * hs[k].x;
        }
        const VT st = from64<VT>(acc);
        w[(int64_t)b * n + i] = st;
        const double2 s2 = to64(st);
        sq = s2.x * s2.x + s2.y * s2.y;
    }
    if (norm2) {
        sq = block_sum(sq);
        if (threadIdx.x == 0) norm2[(int64_t)b * gridDim.x + blockIdx.x] = sq;
    }
}

// out = w / sqrt(norm2[b]) for active items
template <typename VT>
__global__ __launch_bounds__(BT) void scale_kernel(const VT* __restrict__ w, VT* __restrict__ out, int64_t n,
                                                   const double* __restrict__ norm2, const int32_t* __restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const double nrm = sqrt(norm2[b]);
    if (!(nrm > 0.0)) return;
    const double inv = 1.0 / nrm;
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i < n) {
        double2 v = to64(w[(int64_t)b * n + i]);
        v.x *= inv;
        v.y *= inv;
        out[(int64_t)b * n + i] = from64<VT>(v);
    }
}

// g = (beta, 0, ...); clears the rotation state
__global__ void init_cycle_kernel(const double* __restrict__ beta2, double2* __restrict__ g, int batch,
                                  const int32_t* __restrict__ active) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch || !active[b]) return;
    g[b * KMAX] = make_double2(sqrt(beta2[b]), 0.0);
    for (int k = 1; k < KMAX; ++k) g[b * KMAX + k] = make_double2(0.0, 0.0);
}

// One Givens step for column j (one thread per item).  H is column-major
// (KMAX rows per column), cs real cosines, sn complex sines.
__global__ void givens_kernel(double2* __restrict__ H, double* __restrict__ cs, double2* __restrict__ sn,
                              double2* __restrict__ g, const double2* __restrict__ hsum, const double* __restrict__ wn2,
                              int j, int m, int batch, const double* __restrict__ bnorm, double tol,
                              double* __restrict__ est, int32_t* __restrict__ active, int32_t* __restrict__ steps) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch || !active[b]) return;
    double2* col = H + ((int64_t)b * m + j) * KMAX;
    for (int i = 0; i <= j; ++i) col[i] = hsum[b * KMAX + i];
    const double beta = sqrt(wn2[b]);
    col[j + 1] = make_double2(beta, 0.0);
    double* c = cs + (int64_t)b * KMAX;
    double2* s = sn + (int64_t)b * KMAX;
    for (int i = 0; i < j; ++i) {
        const double2 a = col[i], d = col[i + 1];
        // [c s; -conj(s) c] [a; d]
        const double2 t = make_double2(c[i] * a.x + (s[i].x * d.x - s[i].y * d.y), c[i] * a.y + (s[i].x * d.y + s[i].y * d.x));
        const double2 u = make_double2(-(s[i].x * a.x + s[i].y * a.y) + c[i] * d.x, -(s[i].x * a.y - s[i].y * a.x) + c[i] * d.y);
        col[i] = t;
        col[i + 1] = u;
    }
    const double2 a = col[j];
    const double bb = beta;   // real, >= 0
    const double aa = sqrt(a.x * a.x + a.y * a.y);
    double cj;
    double2 sj, r;
    if (bb == 0.0) {
        cj = 1.0; sj = make_double2(0.0, 0.0); r = a;
    } else {
        const double nu = sqrt(aa * aa + bb * bb);
        const double2 ph = aa > 0.0 ? make_double2(a.x / aa, a.y / aa) : make_double2(1.0, 0.0);
        cj = aa / nu;
        sj = make_double2(ph.x * bb / nu, ph.y * bb / nu);   // phase(a) * conj(bb) / nu, bb real
        r = make_double2(ph.x * nu, ph.y * nu);
    }
    c[j] = cj;
    s[j] = sj;
    col[j] = r;
    col[j + 1] = make_double2(0.0, 0.0);
    double2* gb = g + (int64_t)b * KMAX;
    const double2 gj = gb[j];
    gb[j] = make_double2(cj * gj.x, cj * gj.y);
    gb[j + 1] = make_double2(-(sj.x * gj.x + sj.y * gj.y), -(sj.x * gj.y - sj.y * gj.x));   // -conj(s) g_j
    const double e = sqrt(gb[j + 1].x * gb[j + 1].x + gb[j + 1].y * gb[j + 1].y) / bnorm[b];
    est[b] = e;
    steps[b] = j + 1;
    if (!(e > tol) || bb == 0.0 || !(r.x == r.x) || j + 1 >= m) active[b] = 0;
}

// y = R^{-1} g[0..s-1] (one thread per item)
__global__ void backsolve_kernel(const double2* __restrict__ H, const double2* __restrict__ g, int m, int batch,
                                 const int32_t* __restrict__ steps, double2* __restrict__ y,
                                 const int32_t* __restrict__ active) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch || !active[b]) return;
    const int s = steps[b];
    for (int i = s - 1; i >= 0; --i) {
        double2 acc = g[b * KMAX + i];
        for (int k = i + 1; k < s; ++k) {
            const double2 R = H[((int64_t)b * m + k) * KMAX + i];
            const double2 yk = y[b * KMAX + k];
            acc.x -= R.x * yk.x - R.y * yk.y;
            acc.y -= R.x * yk.y + R.y * yk.x;
        }
        const double2 d = H[((int64_t)b * m + i) * KMAX + i];
        const double den = d.x * d.x + d.y * d.y;
        y[b * KMAX + i] = make_double2((acc.x * d.x + acc.y * d.y) / den, (acc.y * d.x - acc.x * d.y) / den);
    }
}

// u = sum_{k < steps[b]} V_k y_k
template <typename VT>
__global__ __launch_bounds__(BT) void combine_kernel(const VT* __restrict__ V, int64_t kstride, int64_t n,
                                                     const double2* __restrict__ y, const int32_t* __restrict__ steps,
                                                     VT* __restrict__ u, const int32_t* __restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    __shared__ double2 ys[KMAX];
    const int s = steps[b];
    for (int k = threadIdx.x; k < s; k += BT) ys[k] = y[b * KMAX + k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    double2 acc = make_double2(0.0, 0.0);
    const VT* Vb = V + (int64_t)b * n + i;
    for (int k = 0; k < s; ++k) {
        const double2 v = to64(Vb[(int64_t)k * kstride]);
        acc.x += v.x * ys[k].x - v.y * ys[k].y;
        acc.y += v.x * ys[k].y + v.y * ys[k].x;
    }
    u[(int64_t)b * n + i] = from64<VT>(acc);
}

// x += alpha[b] * z (alpha = 1 if null), FP64 arithmetic
template <typename XT, typename ZT>
__global__ __launch_bounds__(BT) void axpy_kernel(XT* __restrict__ x, const ZT* __restrict__ z, int64_t n,
                                                  const double* __restrict__ alpha2, const int32_t* __restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    const double a = alpha2 ? sqrt(alpha2[b]) : 1.0;
    double2 xv = to64(x[(int64_t)b * n + i]);
    const double2 zv = to64(z[(int64_t)b * n + i]);
    xv.x += a * zv.x;
    xv.y += a * zv.y;
    x[(int64_t)b * n + i] = from64<XT>(xv);
}

template <typename VT>
__global__ __launch_bounds__(BT) void zero_kernel(VT* __restrict__ x, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i < count) { x[i].x = 0; x[i].y = 0; }
}

// ---------------------------------------------------------------------------------

struct Work {
    int batch = 0, m = 0;
    int64_t n = 0;
    int ntile = 0, nrow_blocks = 0, nres = 0;
    DevBuf<char> V, w, z, r;
    DevBuf<double2> H, sn, g, y, h, hsum, part;
    DevBuf<double> cs, bnorm, beta2, wn2, est, np;
    DevBuf<int32_t> act_cyc, act_arn, steps;
    int32_t* h_act = nullptr;
    double* h_est = nullptr;
    double* h_d = nullptr;
    int32_t* h_steps = nullptr;
    ~Work() {
        if (h_act) (void)hipHostFree(h_act);
        if (h_est) (void)hipHostFree(h_est);
        if (h_d) (void)hipHostFree(h_d);
        if (h_steps) (void)hipHostFree(h_steps);
    }
};

template <typename VT>
static om_status work_alloc(Work& W, const om_csr* A, int m) {
    W.batch = A->batch;
    W.m = m;
    W.n = A->n;
    const int64_t n = A->n, B = A->batch;
    W.ntile = (int)((n + TILE - 1) / TILE);
    W.nrow_blocks = (int)blocks_for(n, BT);
    OM_TRY(residual<VT>(A, 0, nullptr, nullptr, nullptr, nullptr, &W.nres, nullptr, nullptr));
    OM_TRY(W.V.alloc((size_t)(m + 1) * B * n * sizeof(VT)));
    OM_TRY(W.w.alloc((size_t)B * n * sizeof(VT)));
    OM_TRY(W.z.alloc((size_t)B * n * sizeof(VT)));
    OM_TRY(W.r.alloc((size_t)B * n * sizeof(VT)));
    OM_TRY(W.H.alloc((size_t)B * m * KMAX));
    OM_TRY(W.sn.alloc((size_t)B * KMAX));
    OM_TRY(W.cs.alloc((size_t)B * KMAX));
    OM_TRY(W.g.alloc((size_t)B * KMAX));
    OM_TRY(W.y.alloc((size_t)B * KMAX));
    OM_TRY(W.h.alloc((size_t)B * KMAX));
    OM_TRY(W.hsum.alloc((size_t)B * KMAX));
    OM_TRY(W.part.alloc((size_t)B * W.ntile * KMAX));
    const int np = std::max(W.nres, std::max(W.nrow_blocks, 1));
    OM_TRY(W.np.alloc((size_t)B * np));
    OM_TRY(W.bnorm.alloc(B));
    OM_TRY(W.beta2.alloc(B));
    OM_TRY(W.wn2.alloc(B));
    OM_TRY(W.est.alloc(B));
    OM_TRY(W.act_cyc.alloc(B));
    OM_TRY(W.act_arn.alloc(B));
    OM_TRY(W.steps.alloc(B));
    OM_HIP(hipHostMalloc((void**)&W.h_act, B * sizeof(int32_t), hipHostMallocDefault));
    OM_HIP(hipHostMalloc((void**)&W.h_est, B * sizeof(double), hipHostMallocDefault));
    OM_HIP(hipHostMalloc((void**)&W.h_d, 2 * B * sizeof(double), hipHostMallocDefault));
    OM_HIP(hipHostMalloc((void**)&W.h_steps, B * sizeof(int32_t), hipHostMallocDefault));
    return OM_OK;
}

template <typename VT>
static om_status batch_norm2(Work& W, const VT* x, double* out, hipStream_t s) {
    dim3 grid(W.nrow_blocks, W.batch);
    hipLaunchKernelGGL(norm2_partial_kernel<VT>, grid, dim3(BT), 0, s, x, W.n, W.np.p);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(W.batch), dim3(BT), 0, s, W.np.p, W.nrow_blocks, out);
    OM_HIP(hipGetLastError());
    return OM_OK;
}

template <typename VT>
om_status gmres_core(const om_csr* A, const om_ilu* M, int adjoint, const VT* b, VT* x, int m, double tol,
                     int maxiter, const std::vector<int32_t>* item_mask, CoreResult& res, hipStream_t s) {
    constexpr bool C64 = sizeof(VT) == sizeof(float2);
    const int dtype = C64 ? OM_C64 : OM_C128;
    Work W;
    OM_TRY(work_alloc<VT>(W, A, m));
    const int B = A->batch;
    const int64_t n = A->n;
    VT* V = (VT*)W.V.p;
    VT* w = (VT*)W.w.p;
    VT* z = (VT*)W.z.p;
    VT* r = (VT*)W.r.p;
    const int64_t kstride = (int64_t)B * n;

    res.iters.assign(B, 0);
    res.cycles.assign(B, 0);
    res.relres.assign(B, 0.0);
    res.est.assign(B, 0.0);
    res.converged.assign(B, 0);
    std::vector<double> bn(B);
    OM_TRY(batch_norm2<VT>(W, b, W.bnorm.p, s));
    OM_HIP(hipMemcpyAsync(W.h_d, W.bnorm.p, B * sizeof(double), hipMemcpyDeviceToHost, s));
    OM_HIP(hipStreamSynchronize(s));
    std::vector<double> bnorm_h(B);
    for (int i = 0; i < B; ++i) bnorm_h[i] = std::sqrt(W.h_d[i]);
    OM_HIP(hipMemcpyAsync(W.bnorm.p, bnorm_h.data(), B * sizeof(double), hipMemcpyHostToDevice, s));
    std::vector<int32_t> done(B, 0);
    for (int i = 0; i < B; ++i) {
        if (item_mask && !(*item_mask)[i]) done[i] = 2;   // not part of this solve
        if (!done[i] && !(bnorm_h[i] > 0.0)) {         // b = 0: x = 0
            done[i] = 1;
            res.converged[i] = 1;
            if (!std::isfinite(bnorm_h[i])) { set_error("right-hand side is not finite"); return OM_EBREAKDOWN; }
        }
    }
    // zero x for items with b = 0
    for (int i = 0; i < B; ++i)
        if (done[i] == 1) OM_HIP(hipMemsetAsync(x + (int64_t)i * n, 0, n * sizeof(VT), s));

    std::vector<int32_t> act(B);
    while (true) {
        // true residual
        OM_TRY(residual<VT>(A, adjoint, b, x, r, W.np.p, nullptr, nullptr, s, item_mask ? item_mask->data() : nullptr));
        hipLaunchKernelGGL(sum_partials_kernel, dim3(B), dim3(BT), 0, s, W.np.p, W.nres, W.beta2.p);
        OM_HIP(hipMemcpyAsync(W.h_d, W.beta2.p, B * sizeof(double), hipMemcpyDeviceToHost, s));
        OM_HIP(hipStreamSynchronize(s));
        int nact = 0;
        for (int i = 0; i < B; ++i) {
            act[i] = 0;
            if (done[i] == 2) continue;
            const double rr = std::sqrt(W.h_d[i]) / (bnorm_h[i] > 0 ? bnorm_h[i] : 1.0);
            if (done[i] == 1) { res.relres[i] = bnorm_h[i] > 0 ? rr : 0.0; continue; }
            if (!std::isfinite(rr)) { set_error("residual is not finite (item %d)", i); return OM_EBREAKDOWN; }
            res.relres[i] = rr;
            if (rr <= tol) { done[i] = 1; res.converged[i] = 1; continue; }
            if (res.iters[i] >= maxiter) continue;
            act[i] = 1;
            ++nact;
        }
        if (nact == 0) break;
        OM_HIP(hipMemcpyAsync(W.act_cyc.p, act.data(), B * sizeof(int32_t), hipMemcpyHostToDevice, s));
        OM_HIP(hipMemcpyAsync(W.act_arn.p, act.data(), B * sizeof(int32_t), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(init_cycle_kernel, dim3(blocks_for(B, 64)), dim3(64), 0, s, W.beta2.p, W.g.p, B, W.act_cyc.p);
        dim3 vgrid(W.nrow_blocks, B);
        hipLaunchKernelGGL(scale_kernel<VT>, vgrid, dim3(BT), 0, s, r, V, n, W.beta2.p, W.act_cyc.p);
        OM_HIP(hipGetLastError());
        const unsigned ig = blocks_for(B, 64);
        std::vector<int32_t> arn(act);
        int narn = nact;
        for (int j = 0; j < m; ++j) {
            VT* vj = V + (int64_t)j * kstride;
            const VT* zin = vj;
            if (M) {
                OM_TRY(ilu_apply_dev(M, adjoint, dtype, vj, z, W.act_arn.p, s, arn.data()));
                zin = z;
            }
            OM_TRY(spmv<VT>(A, adjoint, zin, w, W.act_arn.p, s, arn.data()));
            dim3 tgrid(W.ntile, B);
            const double vb = (double)narn * (double)n * sizeof(VT);
            for (int pass = 0; pass < 2; ++pass) {
                {
                    ProfScope prof("orth", s, vb * (j + 2));
                    hipLaunchKernelGGL(mdot_kernel<VT>, tgrid, dim3(BT), 0, s, V, kstride, n, j + 1, w, W.part.p,
                                       W.act_arn.p);
                    hipLaunchKernelGGL(mdot_finalize_kernel, dim3(B), dim3(KMAX), 0, s, W.part.p, W.ntile, j + 1, W.h.p,
                                       W.hsum.p, pass, W.act_arn.p);
                }
                ProfScope prof("orth", s, vb * (j + 3));
                hipLaunchKernelGGL(update_kernel<VT>, vgrid, dim3(BT), 0, s, V, kstride, n, j + 1, W.h.p, w,
                                   pass == 1 ? W.np.p : nullptr, W.act_arn.p);
            }
            hipLaunchKernelGGL(sum_partials_kernel, dim3(B), dim3(BT), 0, s, W.np.p, W.nrow_blocks, W.wn2.p);
            hipLaunchKernelGGL(givens_kernel, dim3(ig), dim3(64), 0, s, W.H.p, W.cs.p, W.sn.p, W.g.p, W.hsum.p, W.wn2.p,
                               j, m, B, W.bnorm.p, tol, W.est.p, W.act_arn.p, W.steps.p);
            hipLaunchKernelGGL(scale_kernel<VT>, vgrid, dim3(BT), 0, s, w, V + (int64_t)(j + 1) * kstride, n, W.wn2.p,
                               W.act_arn.p);
            OM_HIP(hipGetLastError());
            OM_HIP(hipMemcpyAsync(W.h_act, W.act_arn.p, B * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            OM_HIP(hipMemcpyAsync(W.h_est, W.est.p, B * sizeof(double), hipMemcpyDeviceToHost, s));
            OM_HIP(hipStreamSynchronize(s));
            if (M) OM_TRY(trsv_check(M, s));
            bool any = false;
            narn = 0;
            for (int i = 0; i < B; ++i) {
                arn[i] = act[i] ? W.h_act[i] : 0;
                narn += arn[i] != 0;
                if (!act[i]) continue;
                res.est[i] = W.h_est[i];
                if (!std::isfinite(W.h_est[i])) { set_error("GMRES breakdown: non-finite residual estimate (item %d)", i); return OM_EBREAKDOWN; }
                if (W.h_act[i]) {
                    if (res.iters[i] + j + 1 >= maxiter) {
                        // stop this item at the iteration limit
                        int32_t zero = 0;
                        OM_HIP(hipMemcpyAsync(W.act_arn.p + i, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
                        OM_HIP(hipStreamSynchronize(s));
                    } else {
                        any = true;
                    }
                }
            }
            if (!any) break;
        }
        // end of cycle
        hipLaunchKernelGGL(backsolve_kernel, dim3(ig), dim3(64), 0, s, W.H.p, W.g.p, m, B, W.steps.p, W.y.p, W.act_cyc.p);
        hipLaunchKernelGGL(combine_kernel<VT>, vgrid, dim3(BT), 0, s, V, kstride, n, W.y.p, W.steps.p, w, W.act_cyc.p);
        const VT* upd = w;
        if (M) {
            OM_TRY(ilu_apply_dev(M, adjoint, dtype, w, z, W.act_cyc.p, s, act.data()));
            upd = z;
        }
        hipLaunchKernelGGL((axpy_kernel<VT, VT>), vgrid, dim3(BT), 0, s, x, upd, n, (const double*)nullptr, W.act_cyc.p);
        OM_HIP(hipGetLastError());
        OM_HIP(hipMemcpyAsync(W.h_steps, W.steps.p, B * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        OM_HIP(hipStreamSynchronize(s));
        if (M) OM_TRY(trsv_check(M, s));
        for (int i = 0; i < B; ++i)
            if (act[i]) {
                res.iters[i] += W.h_steps[i];
                res.cycles[i] += 1;
            }
    }
    return OM_OK;
}

template om_status gmres_core<double2>(const om_csr*, const om_ilu*, int, const double2*, double2*, int, double, int,
                                       const std::vector<int32_t>*, CoreResult&, hipStream_t);
template om_status gmres_core<float2>(const om_csr*, const om_ilu*, int, const float2*, float2*, int, double, int,
                                      const std::vector<int32_t>*, CoreResult&, hipStream_t);

// c64 copy of r / ||r|| for the items in `active`
__global__ __launch_bounds__(BT) void normalise_c64_kernel(const double2* __restrict__ r, float2* __restrict__ out,
                                                           int64_t n, const double* __restrict__ beta2,
                                                           const int32_t* __restrict__ active) {
    const int b = blockIdx.y;
    if (!active[b]) return;
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    const double inv = 1.0 / sqrt(beta2[b]);
    const double2 v = r[(int64_t)b * n + i];
    out[(int64_t)b * n + i] = make_float2((float)(v.x * inv), (float)(v.y * inv));
}

// Mixed-precision GMRES-IR: FP64 residual and update, complex64 inner GMRES.
om_status gmres_ir(const om_csr* A, const om_ilu* M, int adjoint, const double2* b, double2* x, const om_gmres_opts& o,
                   CoreResult& res, int& outer, hipStream_t s) {
    const int B = A->batch;
    const int64_t n = A->n;
    Work W;
    OM_TRY(work_alloc<double2>(W, A, 1));
    DevBuf<float2> rh, d;
    OM_TRY(rh.alloc((size_t)B * n));
    OM_TRY(d.alloc((size_t)B * n));
    DevBuf<double2> r;
    OM_TRY(r.alloc((size_t)B * n));
    OM_TRY(batch_norm2<double2>(W, b, W.bnorm.p, s));
    std::vector<double> bn2(B);
    OM_HIP(hipMemcpyAsync(bn2.data(), W.bnorm.p, B * sizeof(double), hipMemcpyDeviceToHost, s));
    OM_HIP(hipStreamSynchronize(s));
    res.iters.assign(B, 0);
    res.cycles.assign(B, 0);
    res.relres.assign(B, 0.0);
    res.est.assign(B, 0.0);
    res.converged.assign(B, 0);
    std::vector<int32_t> act(B);
    outer = 0;
    const int inner_max = std::max(o.m, 1) * 4;
    while (true) {
        OM_TRY(residual<double2>(A, adjoint, b, x, r.p, W.np.p, nullptr, nullptr, s));
        hipLaunchKernelGGL(sum_partials_kernel, dim3(B), dim3(BT), 0, s, W.np.p, W.nres, W.beta2.p);
        std::vector<double> be2(B);
        OM_HIP(hipMemcpyAsync(be2.data(), W.beta2.p, B * sizeof(double), hipMemcpyDeviceToHost, s));
        OM_HIP(hipStreamSynchronize(s));
        int nact = 0;
        for (int i = 0; i < B; ++i) {
            const double bnrm = std::sqrt(bn2[i]);
            const double rr = bnrm > 0 ? std::sqrt(be2[i]) / bnrm : 0.0;
            if (!std::isfinite(rr)) { set_error("GMRES-IR: residual is not finite (item %d)", i); return OM_EBREAKDOWN; }
            res.relres[i] = rr;
            act[i] = 0;
            if (rr <= o.tol) { res.converged[i] = 1; continue; }
            if (outer >= o.max_outer || res.iters[i] >= o.maxiter) continue;
            act[i] = 1;
            ++nact;
        }
        if (nact == 0) break;
        OM_HIP(hipMemcpyAsync(W.act_cyc.p, act.data(), B * sizeof(int32_t), hipMemcpyHostToDevice, s));
        dim3 vgrid(W.nrow_blocks, B);
        hipLaunchKernelGGL(normalise_c64_kernel, vgrid, dim3(BT), 0, s, r.p, rh.p, n, W.beta2.p, W.act_cyc.p);
        hipLaunchKernelGGL(zero_kernel<float2>, dim3(blocks_for((int64_t)B * n, BT)), dim3(BT), 0, s, d.p, (int64_t)B * n);
        OM_HIP(hipGetLastError());
        CoreResult inner;
        OM_TRY(gmres_core<float2>(A, M, adjoint, rh.p, d.p, o.m, o.inner_tol, inner_max, &act, inner, s));
        hipLaunchKernelGGL((axpy_kernel<double2, float2>), vgrid, dim3(BT), 0, s, x, d.p, n, W.beta2.p, W.act_cyc.p);
        OM_HIP(hipGetLastError());
        for (int i = 0; i < B; ++i)
            if (act[i]) {
                res.iters[i] += inner.iters[i];
                res.cycles[i] += inner.cycles[i];
                res.est[i] = inner.est[i];
            }
        ++outer;
    }
    return OM_OK;
}

}  // namespace omss
