// Preconditioner application: blocked sparse triangular solves on the device.
//
// The factors of an RCM-ordered ILUT have a dependency depth close to n (each
// row reads the one before it), so a level schedule has about one row per
// level.  The solve therefore walks 64-row blocks in order.  For block g:
//   1. every wave of the workgroup takes a share of the ELL slots of the
//      block (entries left of the block, whose unknowns are final) and
//      accumulates sum_j T[r, j] x[j] for its 64 rows (lane = row);
//   2. wave 0 combines the partial sums with the right-hand side and solves
//      the 64x64 unit-lower diagonal block by a column sweep: at step c the
//      finished unknown of lane c is broadcast (readlane) and subtracted from
//      the rows below it.
// One workgroup owns one batch item, so batch items are solved concurrently.
#include "common.hpp"
#include "cplx.hpp"
#include "profile.hpp"

namespace omss {

__device__ inline double bcast(double v, int l) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline float bcast(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

constexpr int TRSV_WAVES = 4;

template <typename VT>
__global__ __launch_bounds__(64 * TRSV_WAVES) void trsv_block_kernel(const TriView<VT>* __restrict__ views, int kind,
                                                                      const VT* rhs, VT* out, int64_t n,
                                                                      const int32_t* __restrict__ active) {
    using ST = typename Scalar<VT>::type;
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    const TriView<VT> S = views[b * 4 + kind];
    const VT* y = rhs + (int64_t)b * n;
    VT* x = out + (int64_t)b * n;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    __shared__ VT part[TRSV_WAVES][64];
    __shared__ VT tri[2016];

    for (int64_t g = 0; g < S.nblk; ++g) {
        for (int t = threadIdx.x; t < 2016; t += 64 * TRSV_WAVES) tri[t] = S.dg[g * 2016 + t];
        VT acc = czero<VT>();
        const int64_t s0 = S.off[g], s1 = S.off[g + 1];
#pragma unroll 4
        for (int64_t s = s0 + wave; s < s1; s += TRSV_WAVES) {
            const int64_t at = s * 64 + lane;
            const int64_t c = S.col[at];
            const VT v = S.val[at];
            const VT xv = x[S.rev ? (n - 1 - c) : c];
            cfma(acc, v, xv);
        }
        part[wave][lane] = acc;
        __syncthreads();
        if (wave == 0) {
            const int64_t row = g * 64 + lane;
            const bool valid = row < n;
            const int64_t mi = S.rev ? (n - 1 - row) : row;
            VT r = czero<VT>();
            if (valid) {
                r = y[mi];
                if (S.dinv) r = cmul(r, S.dinv[row]);
            }
#pragma unroll
            for (int w = 0; w < TRSV_WAVES; ++w) r = csub(r, part[w][lane]);
            for (int c = 0; c < 63; ++c) {
                const ST xr = bcast(r.x, c);
                const ST xi = bcast(r.y, c);
                if (lane > c) {
                    const VT t = tri[c * 63 - (c * (c - 1)) / 2 + (lane - c - 1)];
                    r.x -= t.x * xr;
                    r.x += t.y * xi;
                    r.y -= t.x * xi;
                    r.y -= t.y * xr;
                }
            }
            if (valid) x[mi] = r;
        }
        __syncthreads();
    }
}

// Algorithmic bytes of one triangular solve over the active items: values and
// column indices of the factor, right-hand side read, solution written, and
// the pivot scaling where present.
static double trsv_bytes(const om_ilu* M, int kind, size_t s, const int32_t* act_host) {
    double b = 0.0;
    for (int i = 0; i < M->batch; ++i) {
        if (act_host && !act_host[i]) continue;
        const TriSched& S = M->sched[(size_t)i * 4 + kind];
        b += (double)S.nnz * (double)(s + 4) + 2.0 * (double)S.n * (double)s + (S.has_dinv ? (double)S.n * s : 0.0);
    }
    return b;
}

template <typename VT>
om_status launch_trsv(const om_ilu* M, const TriView<VT>* views, int kind, const VT* rhs, VT* out,
                      const int32_t* active, const int32_t* act_host, hipStream_t s) {
    ProfScope prof("trsv", s, profile_enabled() ? trsv_bytes(M, kind, sizeof(VT), act_host) : 0.0);
    hipLaunchKernelGGL(trsv_block_kernel<VT>, dim3(M->batch), dim3(64 * TRSV_WAVES), 0, s, views, kind, rhs, out, M->n,
                       active);
    OM_HIP(hipGetLastError());
    return OM_OK;
}

// y = (L U)^{-1} x or (L U)^{-H} x for every active batch item; x, y may alias.
om_status ilu_apply_dev(const om_ilu* M, int adjoint, int dtype, const void* x, void* y, const int32_t* active,
                        hipStream_t s, const int32_t* act_host) {
    const int k0 = adjoint ? 2 : 0, k1 = adjoint ? 3 : 1;
    if (dtype == OM_C128) {
        OM_TRY(launch_trsv<double2>(M, M->views64.p, k0, (const double2*)x, (double2*)y, active, act_host, s));
        OM_TRY(launch_trsv<double2>(M, M->views64.p, k1, (const double2*)y, (double2*)y, active, act_host, s));
    } else {
        OM_TRY(launch_trsv<float2>(M, M->views32.p, k0, (const float2*)x, (float2*)y, active, act_host, s));
        OM_TRY(launch_trsv<float2>(M, M->views32.p, k1, (const float2*)y, (float2*)y, active, act_host, s));
    }
    return OM_OK;
}

}  // namespace omss
