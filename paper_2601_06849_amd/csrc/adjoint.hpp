// Host driver of the adjoint (checkpointing in segments of sqrt(N) to N steps).
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

// ---------------------------------------------------------------------------
// Adjoint driver: checkpoints every K steps, each segment replayed once
// ---------------------------------------------------------------------------

// gradient partial-sum arrays of the reverse sweep
enum AdjPart { kPartXg = 0, kPartXw = 1, kPartY = 2, kPartZ = 3, kPartPoint = 4, kAdjParts = 5 };

struct AdjLayout {
    int K = 1, nck = 1;          // segment length and number of checkpoints
    size_t field = 0;            // bytes per padded field
    size_t ck = 0, seg = 0;      // checkpoint and segment states
    // per step of a segment, the stage fields the reverse sweep reads:
    // w1, w2, (3-D: w3, w4,) W, each `field` bytes, kSlotFields per step
    int slot_fields = 0;
    size_t slots = 0;
    size_t Ub = 0, A[4] = {0, 0, 0, 0};
    // gradient slots of the two x adjoint kernels, the y and z adjoint
    // kernels and the pointwise kernel (one per workgroup and component)
    size_t part[kAdjParts] = {0, 0, 0, 0, 0};
    long nslots[kAdjParts] = {0, 0, 0, 0, 0};
    size_t gsum = 0;             // reduced gradient sums [kAdjParts][NC + 1]
    size_t total = 0;
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr long kPointSlots = 2048;   // workgroups of the pointwise adjoint kernel

// Shortest checkpoint segment: ceil(sqrt(N)) steps.
int min_segment(int nsteps) { return std::max(1, int(std::ceil(std::sqrt(double(std::max(nsteps, 1)))))); }

// Layout for segments of K steps (0: the shortest).  The forward work is
// N - K checkpointing steps plus N replayed ones, so K = N is one forward pass.
AdjLayout adjoint_layout(const Plan& pl, int nsteps, int K = 0) {
    AdjLayout L;
    L.K = K > 0 ? std::min(K, std::max(nsteps, 1)) : min_segment(nsteps);
    L.nck = (std::max(nsteps, 1) + L.K - 1) / L.K;
    L.field = pl.lay.field_bytes;
    const int ng = pl.nc + 1;
    const int px = pl.np[0], py = pl.np[1], pz = pl.np[2];
    L.nslots[kPartXg] = long(py) * pz / 16 * pl.nc;
    L.nslots[kPartXw] = L.nslots[kPartXg];
    if (pl.dim == 3) {
        L.nslots[kPartY] = long(px) / 16 * pz * pl.nc;
        L.nslots[kPartZ] = long(px) * py / 16 * pl.nc;
    } else {
        L.nslots[kPartY] = long(px) / 16 * pl.nc;
    }
    L.nslots[kPartPoint] = kPointSlots;
    size_t off = 0;
    L.ck = off;
    off += size_t(L.nck) * L.field;
    L.seg = off;
    off += size_t(L.K) * L.field;
    L.slot_fields = pl.dim == 3 ? 5 : 3;
    L.slots = off;
    off += size_t(L.K) * L.slot_fields * L.field;
    L.Ub = off;
    off += L.field;
    for (int i = 0; i < 4; ++i) {
        L.A[i] = off;
        off += L.field;
    }
    for (int k = 0; k < kAdjParts; ++k) {
        L.part[k] = off;
        off = a256(off + size_t(std::max(L.nslots[k], 1L)) * ng * 8);
    }
    L.gsum = off;
    off = a256(off + kAdjParts * size_t(ng) * 8);
    L.total = off;
    return L;
}

// The longest segment whose layout fits `bytes` (the layout grows with K from
// the shortest segment on); the shortest if none does.
int adjoint_segment_for(const Plan& pl, int nsteps, size_t bytes) {
    int lo = min_segment(nsteps), hi = std::max(nsteps, 1);
    if (adjoint_layout(pl, nsteps, lo).total > bytes) return lo;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (adjoint_layout(pl, nsteps, mid).total <= bytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// LDS of the adjoint tiles: the x kernels hold four and two fields of one
// component, the outer kernel four.
size_t x_adjoint_lds(int NP, size_t elem, bool second) { return x_lds_bytes(NP, second ? 2 : 4, 1, elem); }
size_t outer_adjoint_lds(int NP, size_t elem) { return outer_lds_bytes(NP, 4, 1, elem); }
constexpr size_t kStaticLds = 1024;   // the reduction scratch of add_partials

etd_status adjoint_supported(const Plan& pl) {
    const size_t e = pl.elem;
    // the replayed forward steps keep W from the fused x stage
    if (!x_fused(pl.np[0], pl.nc, e) || x_adjoint_lds(pl.np[0], e, false) + kStaticLds > kMaxLds)
        return fail(ETD_EUNSUPPORTED, "the adjoint x tile exceeds the LDS budget at this size, precision and component count");
    for (int d = 1; d < pl.dim; ++d)
        if (outer_adjoint_lds(pl.np[d], e) + kStaticLds > kMaxLds)
            return fail(ETD_EUNSUPPORTED, "the adjoint outer tile exceeds the LDS budget at this size and precision");
    return ETD_OK;
}

// Two line or column blocks per adjoint tile where its four fields fit
// (each P fragment then feeds twice the MFMAs): up to NP = 128 in FP32 and
// FP64 states.
int adjoint_cb(int NP, size_t elem) {
    return NP <= 128 && x_lds_bytes(NP, 4, 2, elem) + kStaticLds <= kMaxLds ? 2 : 1;
}

template <typename M, int NC, int RB, int CB, int MAXT, bool SECOND>
etd_status launch_xadj_cb(const XAdjArgs& a, long nlines, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = x_lds_bytes(a.NP, SECOND ? 2 : 4, CB, sizeof(T));
    auto k = SECOND ? x_adjoint_w<M, NC, RB, CB, MAXT> : x_adjoint_g<M, NC, RB, CB, MAXT>;
    static std::atomic<size_t> done{0};
    HIP_TRY(set_lds(k, lds, done), "adjoint x LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(nlines / (16 * CB)), unsigned(NC)), dim3(shape_threads(a.NP, RB)), lds, s,
                       a);
    HIP_TRY(hipGetLastError(), "adjoint x launch");
    return ETD_OK;
}

template <typename M, int NC, int RB, int MAXT, bool SECOND>
etd_status launch_xadj_k(const XAdjArgs& a, long nlines, hipStream_t s) {
    if constexpr (RB == 1 && MAXT <= 512) {   // the shape of NP <= 128
        if (adjoint_cb(a.NP, sizeof(typename M::elem)) == 2 && nlines % 32 == 0)
            return launch_xadj_cb<M, NC, RB, 2, MAXT, SECOND>(a, nlines, s);
    }
    return launch_xadj_cb<M, NC, RB, 1, MAXT, SECOND>(a, nlines, s);
}
#define XADJ_K(RB, MAXT, M, NC, SECOND, a, nl, s) launch_xadj_k<M, NC, RB, MAXT, SECOND>(a, nl, s)

// The x adjoint of all components in one kernel (up to NP = 128, the shape
// of one row block per wave, where its registers fit): two line blocks where
// the four fields per component fit in LDS (not for two FP64-state
// components, whose two-block tiles would spill), else one; 0 beyond NP =
// 128 or where not even one fits (the two kernels above then run).  (A joint
// outer adjoint measured no faster: 0.421 -> 0.425 ms per step.)
int adjoint_joint_cb(int NP, int nc, size_t elem) {
    if (NP > 128) return 0;
    if (!(elem == 8 && nc == 2) && x_lds_bytes(NP, 4 * nc, 2, elem) + kStaticLds <= kMaxLds) return 2;
    if (x_lds_bytes(NP, 4 * nc, 1, elem) + kStaticLds <= kMaxLds) return 1;
    return 0;
}

template <typename M, int NC, int RB, int CB, int MAXT>
etd_status launch_xadj_joint_cb(const XAdjArgs& a, long nlines, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = x_lds_bytes(a.NP, 4 * NC, CB, sizeof(T));
    auto k = x_adjoint_joint<M, NC, RB, CB, MAXT>;
    static std::atomic<size_t> done{0};
    HIP_TRY(set_lds(k, lds, done), "joint adjoint x LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(nlines / (16 * CB))), dim3(shape_threads(a.NP, RB)), lds, s, a);
    HIP_TRY(hipGetLastError(), "joint adjoint x launch");
    return ETD_OK;
}

template <typename M, int NC, int RB, int MAXT>
etd_status launch_xadj_joint(const XAdjArgs& a, long nlines, hipStream_t s) {
    if constexpr (RB == 1 && MAXT <= 512) {
        if (adjoint_joint_cb(a.NP, NC, sizeof(typename M::elem)) == 2 && nlines % 32 == 0)
            return launch_xadj_joint_cb<M, NC, RB, 2, MAXT>(a, nlines, s);
        return launch_xadj_joint_cb<M, NC, RB, 1, MAXT>(a, nlines, s);
    } else {
        return fail(ETD_EUNSUPPORTED, "joint adjoint x kernel beyond 128 points");
    }
}
#define XADJJ_K(RB, MAXT, M, NC, a, nl, s) launch_xadj_joint<M, NC, RB, MAXT>(a, nl, s)

// Adjoint tiles hold four fields, so at small extents few workgroups fit per
// CU: one row block per wave up to NP = 128 doubles their waves (the adjoint
// kernels of a 127^3 two-component FP32 step: 0.335 -> 0.296 ms with the
// earlier joint tiles).
#define ADJ_SHAPE(NP, KERNEL, ...) ((NP) <= 128 ? KERNEL(1, 512, __VA_ARGS__) : DISPATCH_SHAPE(NP, KERNEL, __VA_ARGS__))

template <typename M, int NC, bool FIRST, int RB, int CB, int MAXT>
etd_status launch_oadj_cb(OuterAdjArgs a, long nblocks, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = outer_lds_bytes(a.NP, 4, CB, sizeof(T));
    auto k = outer_adjoint<M, NC, FIRST, RB, CB, MAXT>;
    static std::atomic<size_t> done{0};
    HIP_TRY(set_lds(k, lds, done), "adjoint outer LDS attribute");
    a.ncb /= CB;
    hipLaunchKernelGGL(k, dim3(unsigned(nblocks / CB), unsigned(NC)), dim3(shape_threads(a.NP, RB)), lds, s, a);
    HIP_TRY(hipGetLastError(), "adjoint outer launch");
    return ETD_OK;
}

template <typename M, int NC, bool FIRST, int RB, int MAXT>
etd_status launch_oadj_k(const OuterAdjArgs& a, long nblocks, hipStream_t s) {
    if constexpr (RB == 1 && MAXT <= 512) {
        if (adjoint_cb(a.NP, sizeof(typename M::elem)) == 2 && a.ncb % 2 == 0)
            return launch_oadj_cb<M, NC, FIRST, RB, 2, MAXT>(a, nblocks, s);
    }
    return launch_oadj_cb<M, NC, FIRST, RB, 1, MAXT>(a, nblocks, s);
}
#define OADJ_K(RB, MAXT, M, NC, FIRST, a, nb, s) launch_oadj_k<M, NC, FIRST, RB, MAXT>(a, nb, s)

template <typename T>
etd_status copy_f(const T* src, T* dst, long n, hipStream_t s) {
    hipLaunchKernelGGL(copy_field<T>, dim3(2048), dim3(256), 0, s, src, dst, n);
    HIP_TRY(hipGetLastError(), "copy launch");
    return ETD_OK;
}

#define TRY(expr)                          \
    do {                                   \
        const etd_status st_ = (expr);     \
        if (st_ != ETD_OK) return st_;     \
    } while (0)

template <typename M, int NC>
etd_status adjoint_t(const Plan& pl, StageTimer& tm, const void* u0, double t0, int N, const void* ubarN,
                     void* ubar0, double* grad, char* ws, char* aws, const AdjLayout& L, hipStream_t s) {
    typedef typename M::elem T;
    const int px = pl.np[0], py = pl.np[1], pz = pl.np[2];
    const long sc = long(px) * py * pz;
    const long nf = sc * NC;   // elements per field
    const double tau = pl.prob.tau;
    const Dims dm = dims_of(pl);
    const int ng = NC + 1;
    auto F = [&](size_t off) { return reinterpret_cast<T*>(aws + off); };
    T* U = reinterpret_cast<T*>(ws + pl.lay.field[0]);
    T* ck = F(L.ck);
    T* seg = F(L.seg);
    T* Ub = F(L.Ub);
    // stage fields of step i of the segment
    auto slot = [&](int i, int j) { return aws + L.slots + (size_t(i) * L.slot_fields + j) * L.field; };
    T* A[4] = {F(L.A[0]), F(L.A[1]), F(L.A[2]), F(L.A[3])};
    const size_t fe = L.field / sizeof(T);   // elements between consecutive fields
    const T* diag = reinterpret_cast<const T*>(ws + pl.lay.diag);
    const long dstride = long(pl.diag_stride), dcs = long(kDiagSlots) * dstride;
    const double* gtab = reinterpret_cast<const double*>(ws + pl.lay.grad);

    // ---- forward pass: checkpoints every K steps ----
    hipLaunchKernelGGL(pack_field<T>, dim3(2048), dim3(256), 0, s, static_cast<const T*>(u0), U, dm);
    HIP_TRY(hipGetLastError(), "pack launch");
    for (int c = 0; c < L.nck; ++c) {
        TRY(copy_f<T>(U, ck + c * fe, nf, s));
        const int n0 = c * L.K, n1 = std::min(N, n0 + L.K);
        if (c + 1 < L.nck) TRY((run_steps<M, NC>(pl, tm, ws, t0 + n0 * tau, n1 - n0, s)));
    }
    // ---- adjoint state and gradient slots ----
    hipLaunchKernelGGL(pack_field<T>, dim3(2048), dim3(256), 0, s, static_cast<const T*>(ubarN), Ub, dm);
    HIP_TRY(hipGetLastError(), "pack launch");
    for (int k = 0; k < kAdjParts; ++k) {
        hipLaunchKernelGGL(fill_zero, dim3(64), dim3(256), 0, s, reinterpret_cast<double*>(aws + L.part[k]),
                           std::max(L.nslots[k], 1L) * ng);
        HIP_TRY(hipGetLastError(), "fill launch");
    }
    const double inv_dim = 1.0 / pl.dim;

    for (int c = L.nck - 1; c >= 0; --c) {
        const int n0 = c * L.K, n1 = std::min(N, n0 + L.K);
        // replay the segment, keeping every state and every step's stage fields
        TRY(copy_f<T>(ck + c * fe, seg, nf, s));
        for (int i = 0; i < n1 - n0; ++i) {
            char* f[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
            for (int j = 0; j < L.slot_fields; ++j) f[j] = slot(i, j);
            void* out = i + 1 < n1 - n0 ? static_cast<void*>(seg + (i + 1) * fe) : static_cast<void*>(U);
            TRY((replay_step<M, NC>(pl, tm, ws, t0 + (n0 + i) * tau, seg + i * fe, out, f, s)));
        }
        for (int i = n1 - n0 - 1; i >= 0; --i) {
            const int n = n0 + i;
            const double tn = t0 + n * tau, tn1 = t0 + (n + 1) * tau;
            T* Un = seg + i * fe;
            T* w1 = reinterpret_cast<T*>(slot(i, 0));
            T* w2 = reinterpret_cast<T*>(slot(i, 1));
            T* w3 = pl.dim == 3 ? reinterpret_cast<T*>(slot(i, 2)) : w1;
            T* w4 = pl.dim == 3 ? reinterpret_cast<T*>(slot(i, 3)) : w2;
            T* Wf = reinterpret_cast<T*>(slot(i, L.slot_fields - 1));
            // x direction: (a) g and the weights h into A[2], A[3]; (b) wbar, vbar into A[0], A[1]
            XAdjArgs xa{};
            xa.ubar = Ub;
            xa.W = Wf;
            xa.w = w3;
            xa.v = w4;
            xa.g = A[2];
            xa.h = A[3];
            xa.wbar = A[0];
            xa.vbar = A[1];
            xa.P = ws + pl.lay.P[0];
            xa.diag = diag + long(kDiagX1) * dstride;
            xa.diag_sstride = dstride;
            xa.diag_cstride = dcs;
            xa.NP = px;
            xa.sc = sc;
            xa.npy = py;
            xa.tau = tau;
            xa.rxn = rxn_args(pl, ws, tn1);
            xa.grad = GradArgs{gtab, reinterpret_cast<double*>(aws + L.part[kPartXg]), 0, inv_dim};
            if (adjoint_joint_cb(px, NC, sizeof(T)) > 0) {
                TRY(ADJ_SHAPE(px, XADJJ_K, M, NC, xa, long(py) * pz, s));
            } else {
                TRY(ADJ_SHAPE(px, XADJ_K, M, NC, false, xa, long(py) * pz, s));
                xa.grad.partial = reinterpret_cast<double*>(aws + L.part[kPartXw]);
                TRY(ADJ_SHAPE(px, XADJ_K, M, NC, true, xa, long(py) * pz, s));
            }
            // outer directions
            OuterAdjArgs oa{};
            oa.diag_cstride = dcs;
            oa.sc = sc;
            oa.npx = px;
            oa.npy = py;
            oa.dim = pl.dim;
            oa.rxn = rxn_args(pl, ws, tn);
            const T *Lw, *Lv;
            if (pl.dim == 3) {
                oa.a0 = A[0]; oa.a1 = A[1]; oa.f0 = w1; oa.f1 = w2; oa.out0 = A[2]; oa.out1 = A[3];
                oa.P = ws + pl.lay.P[1];
                oa.diag = diag + long(kDiagY) * dstride;
                oa.NP = py; oa.ncb = px / 16; oa.sk = px; oa.sb = long(px) * py;
                oa.grad = GradArgs{gtab, reinterpret_cast<double*>(aws + L.part[kPartY]), 1, inv_dim};
                TRY(ADJ_SHAPE(py, OADJ_K, M, NC, false, oa, long(px / 16) * pz, s));
                oa.a0 = A[2]; oa.a1 = A[3]; oa.f0 = Un; oa.f1 = nullptr; oa.out0 = A[0]; oa.out1 = A[1];
                oa.P = ws + pl.lay.P[2];
                oa.diag = diag + long(kDiagZ) * dstride;
                oa.NP = pz; oa.ncb = px * py / 16; oa.sk = long(px) * py; oa.sb = 0;
                oa.grad = GradArgs{gtab, reinterpret_cast<double*>(aws + L.part[kPartZ]), 2, inv_dim};
                TRY(ADJ_SHAPE(pz, OADJ_K, M, NC, true, oa, long(px) * py / 16, s));
                Lw = A[0];
                Lv = A[1];
            } else {
                oa.a0 = A[0]; oa.a1 = A[1]; oa.f0 = Un; oa.f1 = nullptr; oa.out0 = A[2]; oa.out1 = A[3];
                oa.P = ws + pl.lay.P[1];
                oa.diag = diag + long(kDiagY) * dstride;
                oa.NP = py; oa.ncb = px / 16; oa.sk = px; oa.sb = 0;
                oa.grad = GradArgs{gtab, reinterpret_cast<double*>(aws + L.part[kPartY]), 1, inv_dim};
                TRY(ADJ_SHAPE(py, OADJ_K, M, NC, true, oa, long(px / 16), s));
                Lw = A[2];
                Lv = A[3];
            }
            hipLaunchKernelGGL((add_jt_field<T, NC>), dim3(unsigned(kPointSlots)), dim3(256), 0, s, Un, Lw, Lv, Ub,
                               sc, rxn_args(pl, ws, tn), px, py, reinterpret_cast<double*>(aws + L.part[kPartPoint]));
            HIP_TRY(hipGetLastError(), "adjoint pointwise launch");
        }
    }
    hipLaunchKernelGGL(unpack_field<T>, dim3(2048), dim3(256), 0, s, Ub, static_cast<T*>(ubar0), dm);
    HIP_TRY(hipGetLastError(), "unpack launch");
    double* gs = reinterpret_cast<double*>(aws + L.gsum);
    for (int k = 0; k < kAdjParts; ++k) {
        hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, s, reinterpret_cast<const double*>(aws + L.part[k]),
                           std::max(L.nslots[k], 1L), ng, gs + k * ng);
        HIP_TRY(hipGetLastError(), "gradient reduction launch");
    }
    double host[kAdjParts * 3];
    HIP_TRY(hipMemcpyAsync(host, gs, kAdjParts * ng * sizeof(double), hipMemcpyDeviceToHost, s), "gradient copy");
    HIP_TRY(hipStreamSynchronize(s), "gradient sync");
    for (int k = 0; k < ng; ++k) {
        double t = 0.0;
        for (int j = 0; j < kAdjParts; ++j) t += host[j * ng + k];
        grad[k] = t;
    }
    return ETD_OK;
}

etd_status check_ws(const Plan& pl, const void* ws) {
    if (!ws) return fail(ETD_EWORKSPACE, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(ETD_EWORKSPACE, "workspace must be 256-byte aligned");
    (void)pl;
    return ETD_OK;
}

// Record an event for the start (begin = true) or end of a stage launch.
etd_status timer_mark(StageTimer& t, int kind, bool begin, hipStream_t s) {
    if (!t.on) return ETD_OK;
    if (t.used == t.pool.size()) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e), "timing event create");
        t.pool.push_back(e);
    }
    HIP_TRY(hipEventRecord(t.pool[t.used], s), "timing event record");
    ++t.used;
    if (begin) t.kind.push_back(kind);
    return ETD_OK;
}

}  // namespace
