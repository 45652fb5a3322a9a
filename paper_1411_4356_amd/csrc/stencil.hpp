// Closed-form stencil of the optomechanical Liouvillian (internal).
//
// Row p = l*N + k holds the equation for rho[k, l] (column stacking,
// Eq. (4)); k = ik*nm + jk and l = il*nm + jl (Sec. III ordering).  Slot s
// (0..NSLOT-1) of a row is one candidate entry; the slots are in increasing
// column order.  The value is linear in each of E, g0, g2, kappa,
// Delta/omega_m and Gamma_m (for fixed n_th), so derivatives of L with
// respect to a parameter are the stencil evaluated at a unit parameter set
// with the others zero.
//
// Besides Eq. (1) the Hamiltonian may carry the quadratic ("membrane in the
// middle") coupling g2 (b + b^dag)^2 a^dag a that the paper names as a
// variant its method applies to unchanged (Sec. V); with the truncated b,
// (b + b^dag)^2 has diagonal j + (j + 1 if j + 1 < N_m) and entries
// sqrt(j + 1) sqrt(j + 2) between j and j + 2.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace omss {

constexpr int NSLOT = 16;   // candidate entries of a row

struct DevParams {
    double delta, omega_m, g0, E, kappa, gm, nth, g2;
};

struct Dims {
    int32_t nc, nm, N;
    int64_t n;
};

// Candidate `slot` (0..NSLOT-1) of row p = l*N + k with k = (ik, jk),
// l = (il, jl) already decoded: returns false if the column is outside the
// truncated space; otherwise sets q and the value for parameters P.
__host__ __device__ inline bool stencil_entry_at(int slot, int64_t p, int ik, int jk, int il, int jl, const Dims& d,
                                                 const DevParams& P, int64_t& q, double2& v) {
    const int64_t N = d.N;
    const int nm = d.nm, nc = d.nc;
    switch (slot) {
        case 0:  // bra, cavity down: l' = (il-1, jl); +i E sqrt(il)
            if (il < 1) return false;
            q = p - (int64_t)nm * N; v = make_double2(0.0, P.E * sqrt((double)il)); return true;
        case 1:  // bra, quadratic: l' = (il, jl-2); +i g2 il sqrt(jl-1) sqrt(jl)
            if (jl < 2) return false;
            q = p - 2 * N; v = make_double2(0.0, P.g2 * (double)il * (sqrt((double)(jl - 1)) * sqrt((double)jl))); return true;
        case 2:  // b^dag jump from rho[(ik,jk-1),(il,jl-1)]
            if (jk < 1 || jl < 1) return false;
            q = p - N - 1; v = make_double2(P.gm * P.nth * sqrt((double)jk * (double)jl), 0.0); return true;
        case 3:  // bra, mechanical down: l' = (il, jl-1); +i g0 il sqrt(jl)
            if (jl < 1) return false;
            q = p - N; v = make_double2(0.0, P.g0 * (double)il * sqrt((double)jl)); return true;
        case 4:  // ket, cavity down: k' = (ik-1, jk); -i E sqrt(ik)
            if (ik < 1) return false;
            q = p - nm; v = make_double2(0.0, -P.E * sqrt((double)ik)); return true;
        case 5:  // ket, quadratic: k' = (ik, jk-2); -i g2 ik sqrt(jk-1) sqrt(jk)
            if (jk < 2) return false;
            q = p - 2; v = make_double2(0.0, -P.g2 * (double)ik * (sqrt((double)(jk - 1)) * sqrt((double)jk))); return true;
        case 6:  // ket, mechanical down: k' = (ik, jk-1); -i g0 ik sqrt(jk)
            if (jk < 1) return false;
            q = p - 1; v = make_double2(0.0, -P.g0 * (double)ik * sqrt((double)jk)); return true;
        case 7: {  // diagonal
            const double dk = jk + (jk + 1 < nm ? jk + 1 : 0), dl = jl + (jl + 1 < nm ? jl + 1 : 0);
            const double hk = -P.delta * ik + P.omega_m * jk + P.g2 * ik * dk;
            const double hl = -P.delta * il + P.omega_m * jl + P.g2 * il * dl;
            const double ck = P.kappa * ik + P.gm * (1.0 + P.nth) * jk + (jk < nm - 1 ? P.gm * P.nth * (jk + 1) : 0.0);
            const double cl = P.kappa * il + P.gm * (1.0 + P.nth) * jl + (jl < nm - 1 ? P.gm * P.nth * (jl + 1) : 0.0);
            q = p; v = make_double2(-0.5 * (ck + cl), -(hk - hl)); return true;
        }
        case 8:  // ket, mechanical up: k' = (ik, jk+1); -i g0 ik sqrt(jk+1)
            if (jk + 1 >= nm) return false;
            q = p + 1; v = make_double2(0.0, -P.g0 * (double)ik * sqrt((double)(jk + 1))); return true;
        case 9:  // ket, quadratic: k' = (ik, jk+2); -i g2 ik sqrt(jk+1) sqrt(jk+2)
            if (jk + 2 >= nm) return false;
            q = p + 2; v = make_double2(0.0, -P.g2 * (double)ik * (sqrt((double)(jk + 1)) * sqrt((double)(jk + 2)))); return true;
        case 10:  // ket, cavity up: k' = (ik+1, jk); -i E sqrt(ik+1)
            if (ik + 1 >= nc) return false;
            q = p + nm; v = make_double2(0.0, -P.E * sqrt((double)(ik + 1))); return true;
        case 11:  // bra, mechanical up: l' = (il, jl+1); +i g0 il sqrt(jl+1)
            if (jl + 1 >= nm) return false;
            q = p + N; v = make_double2(0.0, P.g0 * (double)il * sqrt((double)(jl + 1))); return true;
        case 12:  // b jump from rho[(ik,jk+1),(il,jl+1)]
            if (jk + 1 >= nm || jl + 1 >= nm) return false;
            q = p + N + 1; v = make_double2(P.gm * (1.0 + P.nth) * sqrt((double)(jk + 1) * (double)(jl + 1)), 0.0); return true;
        case 13:  // bra, quadratic: l' = (il, jl+2); +i g2 il sqrt(jl+1) sqrt(jl+2)
            if (jl + 2 >= nm) return false;
            q = p + 2 * N; v = make_double2(0.0, P.g2 * (double)il * (sqrt((double)(jl + 1)) * sqrt((double)(jl + 2)))); return true;
        case 14:  // bra, cavity up: l' = (il+1, jl); +i E sqrt(il+1)
            if (il + 1 >= nc) return false;
            q = p + (int64_t)nm * N; v = make_double2(0.0, P.E * sqrt((double)(il + 1))); return true;
        case 15:  // kappa jump from rho[(ik+1,jk),(il+1,jl)]
            if (ik + 1 >= nc || il + 1 >= nc) return false;
            q = p + (int64_t)nm * (N + 1); v = make_double2(P.kappa * sqrt((double)(ik + 1) * (double)(il + 1)), 0.0); return true;
    }
    return false;
}

// The same for row p, decoded here.
__host__ __device__ inline bool stencil_entry(int slot, int64_t p, const Dims& d, const DevParams& P,
                                              int64_t& q, double2& v) {
    const int64_t N = d.N;
    const int64_t l = p / N, k = p - l * N;
    const int ik = (int)(k / d.nm), jk = (int)(k - (int64_t)ik * d.nm);
    const int il = (int)(l / d.nm), jl = (int)(l - (int64_t)il * d.nm);
    return stencil_entry_at(slot, p, ik, jk, il, jl, d, P, q, v);
}

}  // namespace omss
