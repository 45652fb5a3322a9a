// Device assembly of the Liouvillian of Eq. (3) in the Fock basis, column-
// stacked (Eq. (4)), with the trace condition of Eq. (5).
//
// Row p = l*N + k holds the equation for rho[k, l]; k = ik*nm + jk and
// l = il*nm + jl (a = a_c (x) I, b = I (x) b_m, Sec. III).  Each row has at
// most sixteen entries, evaluated in closed form from Eq. (1) and Eq. (3):
//   diagonal        -i (h_k - h_l) - (c_k + c_l) / 2,
//                   h = -Delta i + omega_m j + g2 i D2(j),
//                   D2(j) = j + (j + 1) [j < nm - 1],
//                   c = kappa i + Gamma (1 + n_th) j + Gamma n_th (j + 1) [j < nm - 1]
//   ket side  -i H[k, k'] rho[k', l]  (k' a neighbour of k in H)
//   bra side  +i rho[k, l'] H[l', l]
//   jumps     kappa a rho a^dag, Gamma (1 + n_th) b rho b^dag, Gamma n_th b^dag rho b
// with H[(i,j),(i+-1,j)] = E sqrt(max i), H[(i,j),(i,j+-1)] = g0 i sqrt(max j)
// and, for the quadratic coupling g2 (b + b^dag)^2 a^dag a (Sec. V; zero in
// Eq. (1)), H[(i,j),(i,j+-2)] = g2 i sqrt(m + 1) sqrt(m + 2), m = min(j, j').
// The sixteen candidate columns are, in increasing order,
//   p - nm N, p - 2N, p - N - 1, p - N, p - nm, p - 2, p - 1, p, p + 1, p + 2,
//   p + nm, p + N, p + N + 1, p + 2N, p + nm N, p + nm (N + 1)
// (distinct and increasing for nc >= 2, nm >= 3; with nm = 2 the +-2 columns
// never exist).  An entry is stored when its value is nonzero for at least one
// item of the batch (so g2 = 0 stores none of the quadratic entries).  Row 0
// is rebuilt on the host for the trace condition.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "cplx.hpp"
#include "stencil.hpp"

namespace omss {

__device__ inline bool nonzero(double2 v) { return v.x != 0.0 || v.y != 0.0; }

__global__ void count_kernel(Dims d, const DevParams* P, int batch, int64_t first_row, int32_t* count) {
    const int64_t p = first_row + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.n) return;
    int c = 0;
    for (int s = 0; s < NSLOT; ++s) {
        int64_t q; double2 v;
        if (!stencil_entry(s, p, d, P[0], q, v)) continue;
        bool nz = nonzero(v);
        for (int b = 1; b < batch && !nz; ++b) {
            stencil_entry(s, p, d, P[b], q, v);
            nz = nonzero(v);
        }
        c += nz;
    }
    count[p] = c;
}

__global__ void fill_kernel(Dims d, const DevParams* P, int batch, int64_t first_row, const int32_t* row_ptr,
                            int32_t* col, double2* val, int64_t nnz) {
    const int64_t p = first_row + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.n) return;
    int64_t pos = row_ptr[p];
    for (int s = 0; s < NSLOT; ++s) {
        int64_t q; double2 v;
        if (!stencil_entry(s, p, d, P[0], q, v)) continue;
        bool nz = nonzero(v);
        for (int b = 1; b < batch && !nz; ++b) {
            double2 u;
            stencil_entry(s, p, d, P[b], q, u);
            nz = nonzero(u);
        }
        if (!nz) continue;
        col[pos] = (int32_t)q;
        val[pos] = v;
        for (int b = 1; b < batch; ++b) {
            double2 u;
            stencil_entry(s, p, d, P[b], q, u);
            val[(int64_t)b * nnz + pos] = u;
        }
        ++pos;
    }
}

__global__ void widen_count_kernel(const int32_t* count, int64_t n, int64_t* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = count[i];
}

__global__ void narrow_ptr_kernel(const int64_t* in, int64_t n1, int32_t* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n1) out[i] = (int32_t)in[i];
}

__global__ void to_c64_kernel(const double2* in, float2* out, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

static bool finite_params(const om_params& p) {
    const double v[] = {p.delta, p.omega_m, p.g0, p.E, p.kappa, p.gamma_m, p.n_th, p.g2};
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

double model_weight(const om_params& p) {
    // mean of diag(L): the Hamiltonian part cancels between ket and bra, the
    // dissipative part is -mean_k c_k
    return -0.5 * (p.kappa * (p.nc - 1) + p.gamma_m * (2.0 * p.n_th + 1.0) * (p.nm - 1));
}

om_status validate_params(const om_params* params, int32_t batch) {
    if (!params || batch < 1) { set_error("params is null or batch < 1"); return OM_EINVAL; }
    const om_params& p0 = params[0];
    if (p0.nc < 2 || p0.nm < 2) { set_error("nc and nm must be >= 2 (got %d, %d)", p0.nc, p0.nm); return OM_EINVAL; }
    for (int b = 0; b < batch; ++b) {
        const om_params& p = params[b];
        if (p.nc != p0.nc || p.nm != p0.nm) { set_error("batch items must share nc and nm"); return OM_EINVAL; }
        if (!finite_params(p)) { set_error("non-finite parameter in batch item %d", b); return OM_EINVAL; }
        if (p.kappa < 0 || p.gamma_m < 0 || p.n_th < 0) {
            set_error("kappa, gamma_m and n_th must be >= 0 (item %d)", b);
            return OM_EINVAL;
        }
        if (model_weight(p) == 0.0) { set_error("model without dissipation: the steady state is not unique"); return OM_EINVAL; }
    }
    const int64_t N = (int64_t)p0.nc * p0.nm;
    if (N * N > (int64_t)INT32_MAX) { set_error("n = N^2 exceeds 2^31"); return OM_EINVAL; }
    return OM_OK;
}

static DevParams dev_params(const om_params& p) {
    return DevParams{p.delta, p.omega_m, p.g0, p.E, p.kappa, p.gamma_m, p.n_th, p.g2};
}

om_status assemble(const om_params* params, int32_t batch, int32_t trace_mode, uint32_t flags, om_csr* A,
                   double* w_out, hipStream_t s) {
    OM_TRY(validate_params(params, batch));
    if (trace_mode < OM_TRACE_NONE || trace_mode > OM_TRACE_ADD_ROW0) { set_error("bad trace mode %d", trace_mode); return OM_EINVAL; }
    const om_params& p0 = params[0];
    Dims d{p0.nc, p0.nm, p0.nc * p0.nm, (int64_t)p0.nc * p0.nm * p0.nc * p0.nm};
    const int64_t n = d.n;

    std::vector<DevParams> hp(batch);
    for (int b = 0; b < batch; ++b) hp[b] = dev_params(params[b]);
    DevBuf<DevParams> dp;
    OM_TRY(dp.upload(hp.data(), batch, s));

    // row 0 on the host: the model row, then the trace condition
    std::vector<int64_t> r0col;
    std::vector<std::vector<double2>> r0val(batch);
    for (int sl = 0; sl < NSLOT; ++sl) {
        int64_t q; double2 v;
        if (!stencil_entry(sl, 0, d, hp[0], q, v)) continue;
        bool nz = v.x != 0.0 || v.y != 0.0;
        std::vector<double2> vs(batch);
        vs[0] = v;
        for (int b = 1; b < batch; ++b) {
            stencil_entry(sl, 0, d, hp[b], q, vs[b]);
            nz = nz || vs[b].x != 0.0 || vs[b].y != 0.0;
        }
        if (!nz) continue;
        r0col.push_back(q);
        for (int b = 0; b < batch; ++b) r0val[b].push_back(vs[b]);
    }
    std::vector<double> w(batch);
    for (int b = 0; b < batch; ++b) w[b] = model_weight(params[b]);
    if (trace_mode != OM_TRACE_NONE) {
        // union of the model row (kept for ADD, dropped for REPLACE) and t
        std::vector<int64_t> cols;
        std::vector<std::vector<double2>> vals(batch);
        size_t a = 0;
        const bool keep = trace_mode == OM_TRACE_ADD_ROW0;
        for (int64_t kk = 0; kk < d.N; ++kk) {
            const int64_t tq = kk * (d.N + 1);
            while (keep && a < r0col.size() && r0col[a] < tq) {
                cols.push_back(r0col[a]);
                for (int b = 0; b < batch; ++b) vals[b].push_back(r0val[b][a]);
                ++a;
            }
            cols.push_back(tq);
            for (int b = 0; b < batch; ++b) {
                double2 v = make_double2(w[b], 0.0);
                if (keep && a < r0col.size() && r0col[a] == tq) { v.x += r0val[b][a].x; v.y += r0val[b][a].y; }
                vals[b].push_back(v);
            }
            if (keep && a < r0col.size() && r0col[a] == tq) ++a;
        }
        while (keep && a < r0col.size()) {
            cols.push_back(r0col[a]);
            for (int b = 0; b < batch; ++b) vals[b].push_back(r0val[b][a]);
            ++a;
        }
        r0col.swap(cols);
        r0val.swap(vals);
    }
    if (w_out) for (int b = 0; b < batch; ++b) w_out[b] = w[b];

    DevBuf<int32_t> count;
    OM_TRY(count.alloc(n));
    const int TPB = 256;
    if (n > 1) {
        hipLaunchKernelGGL(count_kernel, dim3(blocks_for(n - 1, TPB)), dim3(TPB), 0, s, d, dp.p, batch, (int64_t)1, count.p);
        OM_HIP(hipGetLastError());
    }
    const int32_t c0 = (int32_t)r0col.size();
    OM_HIP(hipMemcpyAsync(count.p, &c0, sizeof(int32_t), hipMemcpyHostToDevice, s));

    DevBuf<int64_t> cnt64, ptr64;
    OM_TRY(cnt64.alloc(n + 1));
    OM_TRY(ptr64.alloc(n + 1));
    hipLaunchKernelGGL(widen_count_kernel, dim3(blocks_for(n, TPB)), dim3(TPB), 0, s, count.p, n, cnt64.p);
    OM_HIP(hipMemsetAsync(cnt64.p + n, 0, sizeof(int64_t), s));
    size_t tmp_bytes = 0;
    OM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt64.p, ptr64.p, (int)(n + 1), s));
    DevBuf<char> tmp;
    OM_TRY(tmp.alloc(tmp_bytes + 16));
    OM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, cnt64.p, ptr64.p, (int)(n + 1), s));
    int64_t nnz = 0;
    OM_HIP(hipMemcpyAsync(&nnz, ptr64.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    OM_HIP(hipStreamSynchronize(s));
    if (nnz >= (int64_t)INT32_MAX) { set_error("nnz = %lld does not fit 32-bit row pointers", (long long)nnz); return OM_ENOMEM; }

    A->n = n;
    A->nnz = nnz;
    A->batch = batch;
    A->N = d.N;
    OM_TRY(A->row_ptr.alloc(n + 1));
    OM_TRY(A->col.alloc(nnz));
    OM_TRY(A->val.alloc((size_t)batch * nnz));
    hipLaunchKernelGGL(narrow_ptr_kernel, dim3(blocks_for(n + 1, TPB)), dim3(TPB), 0, s, ptr64.p, n + 1, A->row_ptr.p);
    if (n > 1) {
        hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n - 1, TPB)), dim3(TPB), 0, s, d, dp.p, batch, (int64_t)1,
                           A->row_ptr.p, A->col.p, A->val.p, nnz);
        OM_HIP(hipGetLastError());
    }
    // row 0 starts at offset 0
    std::vector<int32_t> c32(r0col.begin(), r0col.end());
    if (c0) {
        OM_HIP(hipMemcpyAsync(A->col.p, c32.data(), c0 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        for (int b = 0; b < batch; ++b)
            OM_HIP(hipMemcpyAsync(A->val.p + (size_t)b * nnz, r0val[b].data(), c0 * sizeof(double2), hipMemcpyHostToDevice, s));
    }
    if (flags & OM_BUILD_C64) {
        OM_TRY(A->val32.alloc((size_t)batch * nnz));
        hipLaunchKernelGGL(to_c64_kernel, dim3(blocks_for((int64_t)batch * nnz, TPB)), dim3(TPB), 0, s, A->val.p,
                           A->val32.p, (int64_t)batch * nnz);
    }
    OM_HIP(hipGetLastError());
    A->has_model = true;
    A->params.assign(params, params + batch);
    A->trace_mode = trace_mode;
    A->w = w;
    A->permuted = false;
    OM_HIP(hipStreamSynchronize(s));   // host vectors above go out of scope
    return OM_OK;
}

om_status make_c64(om_csr* A, hipStream_t s) {
    if (A->val32.p) return OM_OK;
    const int TPB = 256;
    const int64_t cnt = (int64_t)A->batch * A->nnz;
    OM_TRY(A->val32.alloc(cnt));
    hipLaunchKernelGGL(to_c64_kernel, dim3(blocks_for(cnt, TPB)), dim3(TPB), 0, s, A->val.p, A->val32.p, cnt);
    OM_HIP(hipGetLastError());
    return OM_OK;
}

}  // namespace omss
