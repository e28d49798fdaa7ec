// Reverse-mode kernels of one step.
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

// ---------------------------------------------------------------------------
// Adjoint of one step (reverse mode), for the gradient of a loss of U_N with
// respect to U_0, kappa_c and q.  With every Q symmetric and the directions
// commuting, the transpose of the step of Sec. 3.1 is
//   g  = tau Q3x U+bar,           Wbar = U+bar + J(W)^T g,
//   wbar = Q1x Wbar,              vbar = tau Q2x Wbar - g,
//   Ubar = L wbar + J(U)^T L vbar,   L = Q1y Q1z (3-D) or Q1y (2-D),
// and a parameter p enters through d lambda / d p:
//   dLoss/dp += <Wbar, dQ1x w> + tau <Wbar, dQ2x v> + tau <U+bar, dQ3x d>
//             + <wbar, dL U> + <vbar, dL f(U)>,     d = f(W) - v,
// each <a, dQ b> = sum over lines and modes j of (Pa)_j (Pb)_j Q'(tau
// lambda_j) tau d lambda_j / d p.  The x-direction part and the rest of the
// step are two fused kernels; each workgroup accumulates its FP64 partial
// sums [kappa_0 .. kappa_{NC-1}, q] into its own slot (no atomics, so the
// result is repeatable).
// ---------------------------------------------------------------------------

struct GradArgs {
    const double* table;  // derivative weights, [comp][dir][slot][kMaxPadded]
    double* partial;      // this launch's slots, NC + 1 doubles per workgroup
    int dir;              // contracted direction 0/1/2
    double inv_dim;       // d lambda / d q
};

// Block reduction of the lanes' partial sums; adds them into the slot of this
// workgroup (one writer per slot per launch).
template <int NG>
__device__ __forceinline__ void add_partials(double (&acc)[NG], double* partial) {
    __shared__ double red[16][NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        acc[k] = v;
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NG; ++k) red[w][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < NG) {
        double t = 0.0;
        for (int i = 0; i < int(blockDim.x >> 6); ++i) t += red[i][threadIdx.x];
        partial[long(blockIdx.x) * NG + threadIdx.x] += t;
    }
}

struct XAdjArgs {
    const void* ubar;     // U+bar, all components (stride sc)
    const void* W;        // forward W
    const void* w;        // forward w3
    const void* v;        // forward w4
    void* wbar;           // out: Q1x Wbar
    void* vbar;           // out: tau Q2x Wbar - g
    const void* P;
    const void* diag;     // slot X1 of component 0
    long diag_sstride, diag_cstride;
    int NP;
    long sc;
    int npy;
    double tau;
    RxnArgs rxn;          // at t_{n+1}
    GradArgs grad;
};

// x-direction adjoint over 16 lines.  LDS: 8*NC fields [16 lines][NP + pad]:
// ubar, w, v, W (staged), S1 = P ubar, Sw = P w, Sv = P v (own rows), and the
// scaled coefficients; later slots are reused as noted.
template <typename M, int NC, int RB, int MAXT>
__global__ __launch_bounds__(MAXT) void x_adjoint(XAdjArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename M::acc AT;                 // accumulator type of the products
    typedef typename Vec4<AT>::type A4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int UB = 0, WW = NC, VV = 2 * NC, FW = 3 * NC, S1 = 4 * NC, SW = 5 * NC, SV = 6 * NC, GS = 7 * NC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = 16 * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const long line0 = long(blockIdx.x) * 16;
    const void* __restrict__ P = a.P;
    const T tau = T(a.tau);
    const int vpl = NP / VN;
    const T* src[4] = {static_cast<const T*>(a.ubar), static_cast<const T*>(a.w), static_cast<const T*>(a.v),
                       static_cast<const T*>(a.W)};
#pragma unroll 2
    for (int v = tid; v < 16 * vpl; v += blockDim.x) {
        const int j = v / vpl, x = (v - j * vpl) * VN;
        const long gi = line0 * NP + long(v) * VN;
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                *reinterpret_cast<TV*>(R + (f * NC + c) * AST + j * RS + x) =
                    *reinterpret_cast<const TV*>(src[f] + c * a.sc + gi);
    }
    __syncthreads();
    const int rb0 = RB * w;
    auto bfrag_from = [&](int q0) {
        return [&, q0](int q, int k0) { return lds_vec<T, M::KL>(R + (q0 + q) * AST + li * RS + k0); };
    };
    auto at = [&](int q, int r, int e) -> T& { return R[q * AST + li * RS + 16 * (rb0 + r) + M::row(lg, e)]; };
    const T* __restrict__ dg = static_cast<const T*>(a.diag);
    const double* gt = a.grad.table;
    const long gcs = 3L * kGradSlots * kMaxPadded;   // component stride of the weight table

    // ---- S1 = P ubar, Sw = P w, Sv = P v ----
    T4 ub[RB][NC];
    {
        A4 acc[RB][3 * NC];
        zero<AT, RB, 3 * NC>(acc);
        gemm<M, RB, 3 * NC>(P, NP, rb0, li, lg, acc, bfrag_from(0));
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T* d3 = dg + c * a.diag_cstride + 2 * a.diag_sstride + 16 * (rb0 + r);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ub[r][c][e] = at(UB + c, r, e);
                    at(S1 + c, r, e) = acc[r][c][e];
                    at(SW + c, r, e) = acc[r][NC + c][e];
                    at(SV + c, r, e) = acc[r][2 * NC + c][e];
                    at(GS + c, r, e) = d3[M::row(lg, e)] * acc[r][c][e];   // (q3 - 1/2) S1
                }
            }
    }
    __syncthreads();

    // ---- g = tau (ubar/2 + P ((q3 - 1/2) S1)); d = f(W) - v; Wbar = ubar + J(W)^T g ----
    double gacc[NC + 1];
#pragma unroll
    for (int k = 0; k <= NC; ++k) gacc[k] = 0.0;
    T4 g[RB][NC], wb[RB][NC];
    {
        A4 acc[RB][NC];
        zero<AT, RB, NC>(acc);
        gemm<M, RB, NC>(P, NP, rb0, li, lg, acc, bfrag_from(GS));
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                T Wv[NC], F[NC], gg[NC], jt[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    gg[c] = tau * (T(0.5) * ub[r][c][e] + acc[r][c][e]);
                    g[r][c][e] = gg[c];
                    Wv[c] = at(FW + c, r, e);
                }
                const long line = line0 + li;
                const int x = 16 * (rb0 + r) + M::row(lg, e), y = int(line % a.npy), z = int(line / a.npy);
                react<T, NC>(a.rxn, Wv, F, x, y, z);
                react_jt<T, NC>(a.rxn, Wv, gg, jt);
                if (a.rxn.kind == ETD_RXN_AC_MMS) {   // psi(t_{n+1}) depends on kappa and q
                    const double ue = ac_ue(a.rxn, x, y, z) * double(gg[0]);
                    gacc[0] += a.rxn.ac_mu * ue;
                    gacc[NC] += ue;
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    wb[r][c][e] = ub[r][c][e] + jt[c];
                    at(UB + c, r, e) = F[c] - at(VV + c, r, e);   // d, over ubar
                    at(WW + c, r, e) = wb[r][c][e];               // Wbar, over w
                }
            }
    }
    __syncthreads();

    // ---- Sd = P d, S2 = P Wbar; gradient terms; scaled coefficients of S2 ----
    {
        A4 acc[RB][2 * NC];
        zero<AT, RB, 2 * NC>(acc);
        gemm<M, RB, 2 * NC>(P, NP, rb0, li, lg, acc, bfrag_from(UB));
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T* d1 = dg + c * a.diag_cstride + 16 * (rb0 + r);
                const T* d2 = d1 + a.diag_sstride;
                const double* wt = gt + c * gcs + (long(a.grad.dir) * kGradSlots) * kMaxPadded + 16 * (rb0 + r);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = M::row(lg, e);
                    const double sd = acc[r][c][e], s2 = acc[r][NC + c][e];
                    const double t = s2 * double(at(SW + c, r, e)) * wt[kGradRho1 * kMaxPadded + k] +
                                     s2 * double(at(SV + c, r, e)) * wt[kGradRho2 * kMaxPadded + k] +
                                     double(at(S1 + c, r, e)) * sd * wt[kGradRho3 * kMaxPadded + k];
                    gacc[c] += t * wt[kGradMu * kMaxPadded + k];
                    gacc[NC] += t * a.grad.inv_dim;
                    at(VV + c, r, e) = d1[k] * T(s2);   // (q1 - 1) S2, over v
                    at(FW + c, r, e) = d2[k] * T(s2);   // tau (q2 - 1) S2, over W
                }
            }
    }
    __syncthreads();

    // ---- wbar = Wbar + P ((q1 - 1) S2); vbar = -g + tau Wbar + P (tau (q2 - 1) S2) ----
    {
        A4 acc[RB][2 * NC];
        zero<AT, RB, 2 * NC>(acc);
        gemm<M, RB, 2 * NC>(P, NP, rb0, li, lg, acc, bfrag_from(VV));
        T* __restrict__ ow = static_cast<T*>(a.wbar);
        T* __restrict__ ov = static_cast<T*>(a.vbar);
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const long o = c * a.sc + (line0 + li) * NP + 16 * (rb0 + r);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int x = M::row(lg, e);
                    ow[o + x] = wb[r][c][e] + acc[r][c][e];
                    ov[o + x] = -g[r][c][e] + tau * wb[r][c][e] + acc[r][NC + c][e];
                }
            }
    }
    __syncthreads();
    add_partials<NC + 1>(gacc, a.grad.partial);
}

struct OuterAdjArgs {
    const void* a0;       // adjoint inputs (two fields)
    const void* a1;
    const void* f0;       // forward partners: middle: w1, v1; first: U (f(U) formed here)
    const void* f1;
    void* out0;           // Q1 a0, Q1 a1
    void* out1;
    const void* P;
    const void* diag;     // q1 - 1 of this direction, component 0
    long diag_cstride;
    int NP, ncb;
    long sk, sb, sc;
    int npx, npy, dim;
    RxnArgs rxn;          // first: f at t_n
    GradArgs grad;
};

// Adjoint of an outer stage (z or y): the forward stage applied to the two
// adjoint fields, plus the gradient terms <a, dQ1 f> against the forward
// partners.  LDS: 4*NC fields [16 columns][NP + pad]: a0, a1, f0, f1.
template <typename M, int NC, bool FIRST, int RB, int MAXT>
__global__ __launch_bounds__(MAXT) void outer_adjoint(OuterAdjArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename M::acc AT;                 // accumulator type of the products
    typedef typename Vec4<AT>::type A4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int VPR = 16 / VN;
    constexpr int NA = 2 * NC, NF = 4 * NC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = 16 * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const int cb = blockIdx.x % a.ncb;
    const long bt = blockIdx.x / a.ncb;
    const long gbase = bt * a.sb + long(cb) * 16;
    const void* __restrict__ P = a.P;
    const T* a0 = static_cast<const T*>(a.a0);
    const T* a1 = static_cast<const T*>(a.a1);
    const T* f0 = static_cast<const T*>(a.f0);
    const T* f1 = static_cast<const T*>(a.f1);
#pragma unroll 2
    for (int v = tid; v < NP * VPR; v += blockDim.x) {
        const int k = v / VPR, j0 = (v - k * VPR) * VN;
        const long gi = gbase + long(k) * a.sk + j0;
        TV fa[NC], fb[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const TV x0 = *reinterpret_cast<const TV*>(a0 + gi + c * a.sc);
            const TV x1 = *reinterpret_cast<const TV*>(a1 + gi + c * a.sc);
            fa[c] = *reinterpret_cast<const TV*>(f0 + gi + c * a.sc);
            if constexpr (!FIRST) fb[c] = *reinterpret_cast<const TV*>(f1 + gi + c * a.sc);
#pragma unroll
            for (int t = 0; t < VN; ++t) {
                X[c * AST + (j0 + t) * RS + k] = x0[t];
                X[(NC + c) * AST + (j0 + t) * RS + k] = x1[t];
            }
        }
        if constexpr (FIRST) {
#pragma unroll
            for (int t = 0; t < VN; ++t) {
                const int col = cb * 16 + j0 + t;
                int x, y, z;
                if (a.dim == 3) {
                    z = k;
                    y = col / a.npx;
                    x = col - y * a.npx;
                } else {
                    z = 0;
                    y = k;
                    x = col;
                }
                T uu[NC], ff[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) uu[c] = fa[c][t];
                react<T, NC>(a.rxn, uu, ff, x, y, z);
#pragma unroll
                for (int c = 0; c < NC; ++c) fb[c][t] = ff[c];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int t = 0; t < VN; ++t) {
                X[(NA + c) * AST + (j0 + t) * RS + k] = fa[c][t];
                X[(NA + NC + c) * AST + (j0 + t) * RS + k] = fb[c][t];
            }
    }
    __syncthreads();
    const int rb0 = RB * w;
    auto bfrag = [&](int q, int k0) { return lds_vec<T, M::KL>(X + q * AST + li * RS + k0); };
    auto at = [&](int q, int r, int e) -> T& { return X[q * AST + li * RS + 16 * (rb0 + r) + M::row(lg, e)]; };
    const T* __restrict__ dg = static_cast<const T*>(a.diag);
    const double* gt = a.grad.table;
    const long gcs = 3L * kGradSlots * kMaxPadded;
    double gacc[NC + 1];
#pragma unroll
    for (int k = 0; k <= NC; ++k) gacc[k] = 0.0;
    A4 acc[RB][NF];
    T4 res[RB][NA];
    zero<AT, RB, NF>(acc);
    gemm<M, RB, NF>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double* wt = gt + c * gcs + (long(a.grad.dir) * kGradSlots) * kMaxPadded + 16 * (rb0 + r);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = M::row(lg, e);
                const double t = (double(acc[r][c][e]) * acc[r][NA + c][e] +
                                  double(acc[r][NC + c][e]) * acc[r][NA + NC + c][e]) *
                                 wt[kGradRho1 * kMaxPadded + k];
                gacc[c] += t * wt[kGradMu * kMaxPadded + k];
                gacc[NC] += t * a.grad.inv_dim;
            }
        }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) res[r][q][e] = at(q, r, e);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const T* dc = dg + (q % NC) * a.diag_cstride + 16 * (rb0 + r);
#pragma unroll
            for (int e = 0; e < 4; ++e) at(q, r, e) = acc[r][q][e] * dc[M::row(lg, e)];
        }
    __syncthreads();
    A4 acc2[RB][NA];
    zero<AT, RB, NA>(acc2);
    gemm<M, RB, NA>(P, NP, rb0, li, lg, acc2, bfrag);
    T* __restrict__ out0 = static_cast<T*>(a.out0);
    T* __restrict__ out1 = static_cast<T*>(a.out1);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            T* o = (q < NC ? out0 : out1) + (q % NC) * a.sc + gbase + li;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[long(16 * (rb0 + r) + M::row(lg, e)) * a.sk] = res[r][q][e] + acc2[r][q][e];
        }
    __syncthreads();
    add_partials<NC + 1>(gacc, a.grad.partial);
}

// Ubar = A + J(U)^T B over a padded field (all components at each node).
// B is the adjoint of f(t_n, U); where f depends on kappa or q explicitly
// (AC_MMS) the block adds <B, d f / d p> to its gradient slot.
template <typename T, int NC>
__global__ __launch_bounds__(256) void add_jt_field(const T* __restrict__ U, const T* __restrict__ A,
                                                    const T* __restrict__ B, T* __restrict__ out, long npts,
                                                    RxnArgs r, int px, int py, double* partial) {
    if (r.kind == ETD_RXN_AC_MMS) {
        double gacc[NC + 1];
#pragma unroll
        for (int k = 0; k <= NC; ++k) gacc[k] = 0.0;
        for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < npts; i += long(gridDim.x) * blockDim.x) {
            const long yz = i / px;
            const double ue = ac_ue(r, int(i - yz * px), int(yz % py), int(yz / py)) * double(B[i]);
            gacc[0] += r.ac_mu * ue;
            gacc[NC] += ue;
        }
        add_partials<NC + 1>(gacc, partial);
    }
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < npts; i += long(gridDim.x) * blockDim.x) {
        T u[NC], b[NC], jt[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            u[c] = U[c * npts + i];
            b[c] = B[c * npts + i];
        }
        react_jt<T, NC>(r, u, b, jt);
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c * npts + i] = A[c * npts + i] + jt[c];
    }
}

template <typename T>
__global__ void copy_field(const T* __restrict__ src, T* __restrict__ dst, long n) {
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x) dst[i] = src[i];
}

__global__ void fill_zero(double* __restrict__ p, long n) {
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x) p[i] = 0.0;
}

// Sum the workgroup slots (fixed order) into out[NG].
__global__ void sum_partials(const double* __restrict__ part, long nslots, int ng, double* __restrict__ out) {
    __shared__ double sh[256];
    for (int k = 0; k < ng; ++k) {
        double t = 0.0;
        for (long i = threadIdx.x; i < nslots; i += blockDim.x) t += part[i * ng + k];
        sh[threadIdx.x] = t;
        __syncthreads();
        for (int st = blockDim.x / 2; st > 0; st >>= 1) {
            if (int(threadIdx.x) < st) sh[threadIdx.x] += sh[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = sh[0];
        __syncthreads();
    }
}

}  // namespace
