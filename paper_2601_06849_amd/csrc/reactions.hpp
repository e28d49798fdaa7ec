// Pointwise source terms f(t, u) of the examples and workloads, and their
// transposed Jacobians (for the adjoint).
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

// ---------------------------------------------------------------------------
// Reactions (pointwise source terms of the examples and workloads)
// ---------------------------------------------------------------------------

struct RxnArgs {
    int kind;
    double p[4];
    double ac_rate;        // -lam + kappa * sum_d mu_d + q (AC_MMS)
    double ac_mu;          // sum_d mu_d, d psi / d kappa per unit ue (AC_MMS)
    double exp_lt;         // e^{-lam t} at the stage's time (AC_MMS)
    const double* sines;   // [3][kMaxPadded] sin(pi (x_i - lo)/L), 0 on the padding
    double tau;            // the instance's time step (grouped launches form t from it)
};

// Exact solution and psi of the manufactured Allen-Cahn problem at node
// (x, y, z).  psi depends on kappa and q through ac_rate: d psi / d kappa =
// ac_mu ue, d psi / d q = ue.
__device__ __forceinline__ double ac_ue(const RxnArgs& r, int x, int y, int z) {
    return r.exp_lt * r.sines[x] * r.sines[kMaxPadded + y] * r.sines[2 * kMaxPadded + z];
}

__device__ __forceinline__ double ac_psi(const RxnArgs& r, int x, int y, int z) {
    const double ue = ac_ue(r, x, y, z);
    return r.ac_rate * ue - ue * (1.0 - ue * ue);
}

template <typename T>
__device__ __forceinline__ T react1(const RxnArgs& r, T u, int x, int y, int z) {
    switch (r.kind) {
    case ETD_RXN_LINEAR: return T(r.p[0]) * u;
    case ETD_RXN_FISHER: return T(r.p[0]) * u * (T(1) - u);
    case ETD_RXN_ALLEN_CAHN: return u - u * u * u;
    case ETD_RXN_AC_MMS: return u * (T(1) - u * u) + T(ac_psi(r, x, y, z));
    case ETD_RXN_SATURATING: return T(r.p[0]) * u / (T(1) - u);
    default: return T(0);
    }
}

template <typename T>
__device__ __forceinline__ void react2(const RxnArgs& r, T u, T v, T& fu, T& fv) {
    if (r.kind == ETD_RXN_FHN_CUBIC) {
        fu = u * (T(1) - u) * (u - T(r.p[0])) - v;
        fv = T(r.p[1]) * (u - T(r.p[2]) * v);
    } else {
        fu = u - u * u * u / T(3) - v;
        fv = T(r.p[0]) * (u - T(r.p[1]) * v);
    }
}

// Reaction on NC components at one node: f[c] from u[c].
template <typename T, int NC>
__device__ __forceinline__ void react(const RxnArgs& r, const T* u, T* f, int x, int y, int z) {
    if constexpr (NC == 1) {
        f[0] = react1<T>(r, u[0], x, y, z);
    } else {
        react2<T>(r, u[0], u[1], f[0], f[1]);
    }
}

// J(u)^T g: the transposed pointwise Jacobian of the reaction applied to g
// (the adjoint of a perturbation of u; the forcing of AC_MMS does not depend
// on u).
template <typename T, int NC>
__device__ __forceinline__ void react_jt(const RxnArgs& r, const T* u, const T* g, T* out) {
    if constexpr (NC == 1) {
        T d;
        switch (r.kind) {
        case ETD_RXN_LINEAR: d = T(r.p[0]); break;
        case ETD_RXN_FISHER: d = T(r.p[0]) * (T(1) - T(2) * u[0]); break;
        case ETD_RXN_ALLEN_CAHN:
        case ETD_RXN_AC_MMS: d = T(1) - T(3) * u[0] * u[0]; break;
        case ETD_RXN_SATURATING: {
            const T om = T(1) - u[0];
            d = T(r.p[0]) / (om * om);
            break;
        }
        default: d = T(0);
        }
        out[0] = d * g[0];
    } else {
        T fu_u, fu_v, fv_u, fv_v;
        if (r.kind == ETD_RXN_FHN_CUBIC) {
            // fu = u(1-u)(u-a) - v, fv = eps (u - gam v)
            fu_u = (T(-3) * u[0] + T(2) * (T(1) + T(r.p[0]))) * u[0] - T(r.p[0]);
            fu_v = T(-1);
            fv_u = T(r.p[1]);
            fv_v = -T(r.p[1]) * T(r.p[2]);
        } else {
            // fu = u - u^3/3 - v, fv = eps (u - alpha v)
            fu_u = T(1) - u[0] * u[0];
            fu_v = T(-1);
            fv_u = T(r.p[0]);
            fv_v = -T(r.p[0]) * T(r.p[1]);
        }
        out[0] = fu_u * g[0] + fv_u * g[1];
        out[1] = fu_v * g[0] + fv_v * g[1];
    }
}

}  // namespace
