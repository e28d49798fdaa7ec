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
// lambda_j) tau d lambda_j / d p.  Every adjoint kernel handles one component
// per workgroup (blockIdx.y); the reaction couples components only pointwise,
// so the other component enters where a tile is staged.  Each workgroup
// accumulates its FP64 partial sums [kappa_0 .. kappa_{NC-1}, q] into its own
// slot (no atomics, so the result is repeatable).
// ---------------------------------------------------------------------------

struct GradArgs {
    const double* table;  // derivative weights, [comp][dir][slot][kMaxPadded]
    double* partial;      // this launch's slots, NC + 1 doubles per workgroup
    int dir;              // contracted direction 0/1/2
    double inv_dim;       // d lambda / d q
};

// Block reduction of the lanes' partial sums; adds them into slot `slot` of
// the launch (one writer per slot per launch).
template <int NG>
__device__ __forceinline__ void add_partials(double (&acc)[NG], double* partial, long slot) {
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
        partial[slot * NG + threadIdx.x] += t;
    }
}

__device__ __forceinline__ long grid_slot() { return long(blockIdx.y) * gridDim.x + blockIdx.x; }

struct XAdjArgs {
    const void* ubar;     // U+bar (all components, stride sc)
    const void* W;        // forward W
    const void* w;        // forward w3
    const void* v;        // forward w4
    void* g;              // (a) out, (b) in: g = tau Q3x U+bar
    void* h;              // (a) out, (b) in: spectral weights (P w) rho1 + (P v) rho2
    void* wbar;           // (b) out: Q1x Wbar
    void* vbar;           // (b) out: tau Q2x Wbar - g
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

// x-direction adjoint, part (a), component blockIdx.y over 16*CB lines.  LDS:
// 4 fields [16*CB lines][NP + pad]: U+bar, w, v and d = f(W) - v (formed while
// staging), then (q3 - 1/2) P U+bar.  Writes g and the weights
// h = (P w) rho1 + (P v) rho2 that part (b) pairs with P Wbar, and adds the
// <U+bar, dQ3x d> gradient terms.  B fragment qq of a product is field qq / CB,
// line block qq % CB, so each P fragment feeds CB times as many MFMAs.
template <typename M, int NC, int RB, int CB, int MAXT>
__global__ __launch_bounds__(MAXT) void x_adjoint_g(XAdjArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename M::acc AT;
    typedef typename Vec4<AT>::type A4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int NL = 16 * CB;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = NL * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const int c = blockIdx.y;
    const long line0 = long(blockIdx.x) * NL;
    const long cs = c * a.sc;
    const void* __restrict__ P = a.P;
    const T tau = T(a.tau);
    const int vpl = NP / VN;
    const T* ubar = static_cast<const T*>(a.ubar);
    const T* Wf = static_cast<const T*>(a.W);
    const T* wf = static_cast<const T*>(a.w);
    const T* vf = static_cast<const T*>(a.v);
#pragma unroll 2
    for (int v = tid; v < NL * vpl; v += blockDim.x) {
        const int j = v / vpl, x = (v - j * vpl) * VN;
        const long gi = line0 * NP + long(v) * VN;
        const long line = line0 + j;
        const int y = int(line % a.npy), z = int(line / a.npy);
        const TV ub = *reinterpret_cast<const TV*>(ubar + cs + gi);
        const TV ww = *reinterpret_cast<const TV*>(wf + cs + gi);
        const TV vv = *reinterpret_cast<const TV*>(vf + cs + gi);
        TV Wk[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) Wk[k] = *reinterpret_cast<const TV*>(Wf + k * a.sc + gi);
        TV d;
#pragma unroll
        for (int t = 0; t < VN; ++t) {
            T Wv[NC], F[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) Wv[k] = Wk[k][t];
            react<T, NC>(a.rxn, Wv, F, x + t, y, z);
            d[t] = F[c] - vv[t];
        }
        *reinterpret_cast<TV*>(R + j * RS + x) = ub;
        *reinterpret_cast<TV*>(R + AST + j * RS + x) = ww;
        *reinterpret_cast<TV*>(R + 2 * AST + j * RS + x) = vv;
        *reinterpret_cast<TV*>(R + 3 * AST + j * RS + x) = d;
    }
    __syncthreads();
    const int rb0 = RB * w;
    auto bfrag = [&](int qq, int k0) {
        return lds_vec<T, M::KL>(R + (qq / CB) * AST + ((qq % CB) * 16 + li) * RS + k0);
    };
    auto at = [&](int qq, int r, int e) -> T& {
        return R[(qq / CB) * AST + ((qq % CB) * 16 + li) * RS + 16 * (rb0 + r) + M::row(lg, e)];
    };
    const T* __restrict__ d3 = static_cast<const T*>(a.diag) + c * a.diag_cstride + 2 * a.diag_sstride;
    const double* wt = a.grad.table + c * (3L * kGradSlots * kMaxPadded) + (long(a.grad.dir) * kGradSlots) * kMaxPadded;
    double gacc[NC + 1];
#pragma unroll
    for (int k = 0; k <= NC; ++k) gacc[k] = 0.0;

    // ---- S1 = P U+bar, Sw = P w, Sv = P v, Sd = P d ----
    T4 ub[RB][CB];
    {
        A4 acc[RB][4 * CB];
        zero<AT, RB, 4 * CB>(acc);
        gemm<M, RB, 4 * CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            T* __restrict__ ho = static_cast<T*>(a.h) + cs + (line0 + 16 * b + li) * NP + 16 * rb0;
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 16 * (rb0 + r) + M::row(lg, e);
                    ub[r][b][e] = at(b, r, e);
                    const double t3 = double(acc[r][b][e]) * double(acc[r][3 * CB + b][e]) *
                                      wt[kGradRho3 * kMaxPadded + k];
                    gacc[c] += t3 * wt[kGradMu * kMaxPadded + k];
                    gacc[NC] += t3 * a.grad.inv_dim;
                    ho[16 * r + M::row(lg, e)] = T(double(acc[r][CB + b][e]) * wt[kGradRho1 * kMaxPadded + k] +
                                                   double(acc[r][2 * CB + b][e]) * wt[kGradRho2 * kMaxPadded + k]);
                }
        }
        __syncthreads();
        // (q3 - 1/2) S1 over U+bar
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) at(b, r, e) = d3[16 * (rb0 + r) + M::row(lg, e)] * acc[r][b][e];
    }
    __syncthreads();

    // ---- g = tau (U+bar / 2 + P ((q3 - 1/2) S1)) ----
    A4 acc[RB][CB];
    zero<AT, RB, CB>(acc);
    gemm<M, RB, CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
    for (int b = 0; b < CB; ++b) {
        const long line = line0 + 16 * b + li;
        T* __restrict__ go = static_cast<T*>(a.g) + cs + line * NP + 16 * rb0;
        const int y = int(line % a.npy), z = int(line / a.npy);
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const T gg = tau * (T(0.5) * ub[r][b][e] + acc[r][b][e]);
                go[16 * r + M::row(lg, e)] = gg;
                if (a.rxn.kind == ETD_RXN_AC_MMS) {   // psi(t_{n+1}) depends on kappa and q
                    const double ue = ac_ue(a.rxn, 16 * (rb0 + r) + M::row(lg, e), y, z) * double(gg);
                    gacc[0] += a.rxn.ac_mu * ue;
                    gacc[NC] += ue;
                }
            }
    }
    add_partials<NC + 1>(gacc, a.grad.partial, grid_slot());
}

// x-direction adjoint, part (b), component blockIdx.y over 16*CB lines.  LDS:
// 2 fields: Wbar = U+bar + J(W)^T g (formed while staging), then the scaled
// coefficients (q1 - 1) P Wbar and tau (q2 - 1) P Wbar.  Adds the
// <Wbar, dQ1x w> + tau <Wbar, dQ2x v> gradient terms and writes
// wbar = Q1x Wbar and vbar = tau Q2x Wbar - g.
template <typename M, int NC, int RB, int CB, int MAXT>
__global__ __launch_bounds__(MAXT) void x_adjoint_w(XAdjArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename M::acc AT;
    typedef typename Vec4<AT>::type A4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int NL = 16 * CB;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = NL * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const int c = blockIdx.y;
    const long line0 = long(blockIdx.x) * NL;
    const long cs = c * a.sc;
    const void* __restrict__ P = a.P;
    const T tau = T(a.tau);
    const int vpl = NP / VN;
    const T* ubar = static_cast<const T*>(a.ubar);
    const T* Wf = static_cast<const T*>(a.W);
    const T* gf = static_cast<const T*>(a.g);
#pragma unroll 2
    for (int v = tid; v < NL * vpl; v += blockDim.x) {
        const int j = v / vpl, x = (v - j * vpl) * VN;
        const long gi = line0 * NP + long(v) * VN;
        const TV ub = *reinterpret_cast<const TV*>(ubar + cs + gi);
        TV Wk[NC], gk[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            Wk[k] = *reinterpret_cast<const TV*>(Wf + k * a.sc + gi);
            gk[k] = *reinterpret_cast<const TV*>(gf + k * a.sc + gi);
        }
        TV wb;
#pragma unroll
        for (int t = 0; t < VN; ++t) {
            T Wv[NC], gg[NC], jt[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                Wv[k] = Wk[k][t];
                gg[k] = gk[k][t];
            }
            react_jt<T, NC>(a.rxn, Wv, gg, jt);
            wb[t] = ub[t] + jt[c];
        }
        *reinterpret_cast<TV*>(R + j * RS + x) = wb;
    }
    __syncthreads();
    const int rb0 = RB * w;
    auto bfrag = [&](int qq, int k0) {
        return lds_vec<T, M::KL>(R + (qq / CB) * AST + ((qq % CB) * 16 + li) * RS + k0);
    };
    auto at = [&](int qq, int r, int e) -> T& {
        return R[(qq / CB) * AST + ((qq % CB) * 16 + li) * RS + 16 * (rb0 + r) + M::row(lg, e)];
    };
    const T* __restrict__ d1 = static_cast<const T*>(a.diag) + c * a.diag_cstride;
    const T* __restrict__ d2 = d1 + a.diag_sstride;
    const double* wt = a.grad.table + c * (3L * kGradSlots * kMaxPadded) + (long(a.grad.dir) * kGradSlots) * kMaxPadded;
    double gacc[NC + 1];
#pragma unroll
    for (int k = 0; k <= NC; ++k) gacc[k] = 0.0;

    // ---- S2 = P Wbar; gradient terms against h; scaled coefficients ----
    T4 wb[RB][CB];
    {
        A4 acc[RB][CB];
        zero<AT, RB, CB>(acc);
        gemm<M, RB, CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const T* __restrict__ hi = static_cast<const T*>(a.h) + cs + (line0 + 16 * b + li) * NP + 16 * rb0;
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 16 * (rb0 + r) + M::row(lg, e);
                    wb[r][b][e] = at(b, r, e);
                    const double t = double(acc[r][b][e]) * double(hi[16 * r + M::row(lg, e)]);
                    gacc[c] += t * wt[kGradMu * kMaxPadded + k];
                    gacc[NC] += t * a.grad.inv_dim;
                }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 16 * (rb0 + r) + M::row(lg, e);
                    at(b, r, e) = d1[k] * acc[r][b][e];        // (q1 - 1) S2
                    at(CB + b, r, e) = d2[k] * acc[r][b][e];   // tau (q2 - 1) S2
                }
    }
    __syncthreads();

    // ---- wbar = Wbar + P ((q1 - 1) S2); vbar = -g + tau Wbar + P (tau (q2 - 1) S2) ----
    A4 acc[RB][2 * CB];
    zero<AT, RB, 2 * CB>(acc);
    gemm<M, RB, 2 * CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
    for (int b = 0; b < CB; ++b) {
        const long o = cs + (line0 + 16 * b + li) * NP + 16 * rb0;
        T* __restrict__ ow = static_cast<T*>(a.wbar) + o;
        T* __restrict__ ov = static_cast<T*>(a.vbar) + o;
        const T* __restrict__ gi = gf + o;
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = 16 * r + M::row(lg, e);
                ow[x] = wb[r][b][e] + acc[r][b][e];
                ov[x] = -gi[x] + tau * wb[r][b][e] + acc[r][CB + b][e];
            }
    }
    add_partials<NC + 1>(gacc, a.grad.partial, grid_slot());
}

// x-direction adjoint of every component of 16*CB lines in one workgroup,
// where the 4*NC fields fit in LDS: parts (a) and (b) above with g, Wbar and
// the weights h kept on chip (no round trip through memory, and each P
// fragment feeds the products of all components).  LDS: field f*NC + c of
// component c, f = 0 (U+bar, then (q3 - 1/2) P U+bar, then Wbar, then
// (q1 - 1) P Wbar), 1 (w, then tau (q2 - 1) P Wbar), 2 (v), 3 (d = f(W) - v).
// The gradient partials go to the slots of part (a).
template <typename M, int NC, int RB, int CB, int MAXT>
__global__ __launch_bounds__(MAXT) void x_adjoint_joint(XAdjArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename M::acc AT;
    typedef typename Vec4<AT>::type A4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int NL = 16 * CB;
    constexpr int NF = 4 * NC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = NL * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const long line0 = long(blockIdx.x) * NL;
    const void* __restrict__ P = a.P;
    const T tau = T(a.tau);
    const int vpl = NP / VN;
    const T* ubar = static_cast<const T*>(a.ubar);
    const T* Wf = static_cast<const T*>(a.W);
    const T* wf = static_cast<const T*>(a.w);
    const T* vf = static_cast<const T*>(a.v);
#pragma unroll 2
    for (int v = tid; v < NL * vpl; v += blockDim.x) {
        const int j = v / vpl, x = (v - j * vpl) * VN;
        const long gi = line0 * NP + long(v) * VN;
        const long line = line0 + j;
        const int y = int(line % a.npy), z = int(line / a.npy);
        TV Wk[NC], vv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            Wk[c] = *reinterpret_cast<const TV*>(Wf + c * a.sc + gi);
            vv[c] = *reinterpret_cast<const TV*>(vf + c * a.sc + gi);
            *reinterpret_cast<TV*>(R + c * AST + j * RS + x) = *reinterpret_cast<const TV*>(ubar + c * a.sc + gi);
            *reinterpret_cast<TV*>(R + (NC + c) * AST + j * RS + x) = *reinterpret_cast<const TV*>(wf + c * a.sc + gi);
            *reinterpret_cast<TV*>(R + (2 * NC + c) * AST + j * RS + x) = vv[c];
        }
        TV d[NC];
#pragma unroll
        for (int t = 0; t < VN; ++t) {
            T Wv[NC], F[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) Wv[c] = Wk[c][t];
            react<T, NC>(a.rxn, Wv, F, x + t, y, z);
#pragma unroll
            for (int c = 0; c < NC; ++c) d[c][t] = F[c] - vv[c][t];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) *reinterpret_cast<TV*>(R + (3 * NC + c) * AST + j * RS + x) = d[c];
    }
    __syncthreads();
    const int rb0 = RB * w;
    auto bfrag = [&](int qq, int k0) {
        return lds_vec<T, M::KL>(R + (qq / CB) * AST + ((qq % CB) * 16 + li) * RS + k0);
    };
    auto at = [&](int f, int b, int r, int e) -> T& {
        return R[f * AST + (b * 16 + li) * RS + 16 * (rb0 + r) + M::row(lg, e)];
    };
    auto wt = [&](int c) {
        return a.grad.table + c * (3L * kGradSlots * kMaxPadded) + (long(a.grad.dir) * kGradSlots) * kMaxPadded;
    };
    auto dslot = [&](int c, int slot) {
        return static_cast<const T*>(a.diag) + c * a.diag_cstride + slot * a.diag_sstride;
    };
    double gacc[NC + 1];
#pragma unroll
    for (int k = 0; k <= NC; ++k) gacc[k] = 0.0;

    // ---- S1 = P U+bar, Sw = P w, Sv = P v, Sd = P d of every component ----
    T4 ub[RB][NC][CB], h[RB][NC][CB];
    {
        A4 acc[RB][NF * CB];
        zero<AT, RB, NF * CB>(acc);
        gemm<M, RB, NF * CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double* wc = wt(c);
#pragma unroll
            for (int b = 0; b < CB; ++b)
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int k = 16 * (rb0 + r) + M::row(lg, e);
                        ub[r][c][b][e] = at(c, b, r, e);
                        const double t3 = double(acc[r][c * CB + b][e]) * double(acc[r][(3 * NC + c) * CB + b][e]) *
                                          wc[kGradRho3 * kMaxPadded + k];
                        gacc[c] += t3 * wc[kGradMu * kMaxPadded + k];
                        gacc[NC] += t3 * a.grad.inv_dim;
                        h[r][c][b][e] = T(double(acc[r][(NC + c) * CB + b][e]) * wc[kGradRho1 * kMaxPadded + k] +
                                          double(acc[r][(2 * NC + c) * CB + b][e]) * wc[kGradRho2 * kMaxPadded + k]);
                    }
        }
        __syncthreads();
        // (q3 - 1/2) S1 over U+bar
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const T* d3 = dslot(c, 2);
#pragma unroll
            for (int b = 0; b < CB; ++b)
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        at(c, b, r, e) = d3[16 * (rb0 + r) + M::row(lg, e)] * acc[r][c * CB + b][e];
        }
    }
    __syncthreads();

    // ---- g = tau (U+bar / 2 + P ((q3 - 1/2) S1)); Wbar = U+bar + J(W)^T g ----
    T4 wb[RB][NC][CB], g[RB][NC][CB];
    {
        A4 acc[RB][NC * CB];
        zero<AT, RB, NC * CB>(acc);
        gemm<M, RB, NC * CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const long line = line0 + 16 * b + li;
            const int y = int(line % a.npy), z = int(line / a.npy);
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int x = 16 * (rb0 + r) + M::row(lg, e);
                    T Wv[NC], gg[NC], jt[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        gg[c] = tau * (T(0.5) * ub[r][c][b][e] + acc[r][c * CB + b][e]);
                        g[r][c][b][e] = gg[c];
                        Wv[c] = Wf[c * a.sc + line * NP + x];
                    }
                    if (a.rxn.kind == ETD_RXN_AC_MMS) {   // psi(t_{n+1}) depends on kappa and q
                        const double ue = ac_ue(a.rxn, x, y, z) * double(gg[0]);
                        gacc[0] += a.rxn.ac_mu * ue;
                        gacc[NC] += ue;
                    }
                    react_jt<T, NC>(a.rxn, Wv, gg, jt);
#pragma unroll
                    for (int c = 0; c < NC; ++c) wb[r][c][b][e] = ub[r][c][b][e] + jt[c];
                }
        }
    }
    __syncthreads();   // every wave has read (q3 - 1/2) S1
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) at(c, b, r, e) = wb[r][c][b][e];
    __syncthreads();

    // ---- S2 = P Wbar; gradient terms against h; scaled coefficients ----
    {
        A4 acc[RB][NC * CB];
        zero<AT, RB, NC * CB>(acc);
        gemm<M, RB, NC * CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double* wc = wt(c);
#pragma unroll
            for (int b = 0; b < CB; ++b)
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int k = 16 * (rb0 + r) + M::row(lg, e);
                        const double t = double(acc[r][c * CB + b][e]) * double(h[r][c][b][e]);
                        gacc[c] += t * wc[kGradMu * kMaxPadded + k];
                        gacc[NC] += t * a.grad.inv_dim;
                    }
        }
        __syncthreads();   // every wave has read Wbar
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const T* d1 = dslot(c, 0);
            const T* d2 = dslot(c, 1);
#pragma unroll
            for (int b = 0; b < CB; ++b)
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int k = 16 * (rb0 + r) + M::row(lg, e);
                        at(c, b, r, e) = d1[k] * acc[r][c * CB + b][e];        // (q1 - 1) S2
                        at(NC + c, b, r, e) = d2[k] * acc[r][c * CB + b][e];   // tau (q2 - 1) S2
                    }
        }
    }
    __syncthreads();

    // ---- wbar = Wbar + P ((q1 - 1) S2); vbar = -g + tau Wbar + P (tau (q2 - 1) S2) ----
    A4 acc[RB][2 * NC * CB];
    zero<AT, RB, 2 * NC * CB>(acc);
    gemm<M, RB, 2 * NC * CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const long o = c * a.sc + (line0 + 16 * b + li) * NP + 16 * rb0;
            T* __restrict__ ow = static_cast<T*>(a.wbar) + o;
            T* __restrict__ ov = static_cast<T*>(a.vbar) + o;
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int x = 16 * r + M::row(lg, e);
                    ow[x] = wb[r][c][b][e] + acc[r][c * CB + b][e];
                    ov[x] = -g[r][c][b][e] + tau * wb[r][c][b][e] + acc[r][(NC + c) * CB + b][e];
                }
        }
    add_partials<NC + 1>(gacc, a.grad.partial, grid_slot());
}

struct OuterAdjArgs {
    const void* a0;       // adjoint inputs (two fields, all components)
    const void* a1;
    const void* f0;       // forward partners: middle: w1, w2; first: U (f(U) formed here)
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

// Adjoint of an outer stage (z or y) for component blockIdx.y: the forward
// stage applied to the two adjoint fields, plus the gradient terms
// <a, dQ1 f> against the forward partners.  LDS: 4 fields [16*CB columns][NP +
// pad]: a0, a1, f0, f1; B fragment qq is field qq / CB, column block qq % CB.
// a.ncb counts tiles of 16*CB columns per batch.
template <typename M, int NC, bool FIRST, int RB, int CB, int MAXT>
__global__ __launch_bounds__(MAXT) void outer_adjoint(OuterAdjArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename M::acc AT;
    typedef typename Vec4<AT>::type A4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int NCOL = 16 * CB;
    constexpr int VPR = NCOL / VN;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = NCOL * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const int c = blockIdx.y;
    const long cs = c * a.sc;
    const int cb = blockIdx.x % a.ncb;
    const long bt = blockIdx.x / a.ncb;
    const long gbase = bt * a.sb + long(cb) * NCOL;
    const void* __restrict__ P = a.P;
    const T* a0 = static_cast<const T*>(a.a0);
    const T* a1 = static_cast<const T*>(a.a1);
    const T* f0 = static_cast<const T*>(a.f0);
    const T* f1 = static_cast<const T*>(a.f1);
#pragma unroll 2
    for (int v = tid; v < NP * VPR; v += blockDim.x) {
        const int k = v / VPR, j0 = (v - k * VPR) * VN;
        const long gi = gbase + long(k) * a.sk + j0;
        const TV x0 = *reinterpret_cast<const TV*>(a0 + cs + gi);
        const TV x1 = *reinterpret_cast<const TV*>(a1 + cs + gi);
        TV fa, fb;
        if constexpr (FIRST) {
            TV uk[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) uk[q] = *reinterpret_cast<const TV*>(f0 + q * a.sc + gi);
            fa = uk[c];
#pragma unroll
            for (int t = 0; t < VN; ++t) {
                const int col = cb * NCOL + j0 + t;
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
                for (int q = 0; q < NC; ++q) uu[q] = uk[q][t];
                react<T, NC>(a.rxn, uu, ff, x, y, z);
                fb[t] = ff[c];
            }
        } else {
            fa = *reinterpret_cast<const TV*>(f0 + cs + gi);
            fb = *reinterpret_cast<const TV*>(f1 + cs + gi);
        }
#pragma unroll
        for (int t = 0; t < VN; ++t) {
            X[(j0 + t) * RS + k] = x0[t];
            X[AST + (j0 + t) * RS + k] = x1[t];
            X[2 * AST + (j0 + t) * RS + k] = fa[t];
            X[3 * AST + (j0 + t) * RS + k] = fb[t];
        }
    }
    __syncthreads();
    const int rb0 = RB * w;
    auto bfrag = [&](int qq, int k0) {
        return lds_vec<T, M::KL>(X + (qq / CB) * AST + ((qq % CB) * 16 + li) * RS + k0);
    };
    auto at = [&](int qq, int r, int e) -> T& {
        return X[(qq / CB) * AST + ((qq % CB) * 16 + li) * RS + 16 * (rb0 + r) + M::row(lg, e)];
    };
    const T* __restrict__ dc = static_cast<const T*>(a.diag) + c * a.diag_cstride;
    const double* wt = a.grad.table + c * (3L * kGradSlots * kMaxPadded) + (long(a.grad.dir) * kGradSlots) * kMaxPadded;
    double gacc[NC + 1];
#pragma unroll
    for (int k = 0; k <= NC; ++k) gacc[k] = 0.0;
    T4 res[RB][2 * CB];
    {
        A4 acc[RB][4 * CB];
        zero<AT, RB, 4 * CB>(acc);
        gemm<M, RB, 4 * CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 16 * (rb0 + r) + M::row(lg, e);
                    const double t = (double(acc[r][b][e]) * acc[r][2 * CB + b][e] +
                                      double(acc[r][CB + b][e]) * acc[r][3 * CB + b][e]) *
                                     wt[kGradRho1 * kMaxPadded + k];
                    gacc[c] += t * wt[kGradMu * kMaxPadded + k];
                    gacc[NC] += t * a.grad.inv_dim;
                    res[r][b][e] = at(b, r, e);
                    res[r][CB + b][e] = at(CB + b, r, e);
                }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const T d = dc[16 * (rb0 + r) + M::row(lg, e)];
                    at(b, r, e) = acc[r][b][e] * d;
                    at(CB + b, r, e) = acc[r][CB + b][e] * d;
                }
    }
    __syncthreads();
    A4 acc[RB][2 * CB];
    zero<AT, RB, 2 * CB>(acc);
    gemm<M, RB, 2 * CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
    for (int b = 0; b < CB; ++b) {
        T* __restrict__ o0 = static_cast<T*>(a.out0) + cs + gbase + 16 * b + li;
        T* __restrict__ o1 = static_cast<T*>(a.out1) + cs + gbase + 16 * b + li;
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long row = long(16 * (rb0 + r) + M::row(lg, e)) * a.sk;
                o0[row] = res[r][b][e] + acc[r][b][e];
                o1[row] = res[r][CB + b][e] + acc[r][CB + b][e];
            }
    }
    add_partials<NC + 1>(gacc, a.grad.partial, grid_slot());
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
        add_partials<NC + 1>(gacc, partial, blockIdx.x);
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
