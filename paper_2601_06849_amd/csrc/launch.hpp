// Host-side launch plumbing: tile shapes, launchers and the step drivers.
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

// ---------------------------------------------------------------------------
// Host-side launch plumbing
// ---------------------------------------------------------------------------

Dims dims_of(const Plan& p) {
    Dims d;
    d.nc = p.nc;
    d.nx = p.n[0];
    d.ny = p.n[1];
    d.nz = p.n[2];
    d.px = p.np[0];
    d.py = p.np[1];
    d.pz = p.np[2];
    return d;
}

RxnArgs rxn_args(const Plan& pl, const char* ws, double t) {
    const etd_problem& p = pl.prob;
    RxnArgs r;
    r.kind = p.rxn;
    for (int i = 0; i < 4; ++i) r.p[i] = p.rxn_param[i];
    r.sines = reinterpret_cast<const double*>(ws + pl.lay.sines);
    r.ac_rate = 0.0;
    r.ac_mu = 0.0;
    r.exp_lt = 0.0;
    r.tau = p.tau;
    if (p.rxn == ETD_RXN_AC_MMS) {
        const double lam = p.rxn_param[0];
        double mu = 0.0;
        for (int d = 0; d < p.dim; ++d) {
            const double L = p.hi[d] - p.lo[d];
            if (p.rxn_param[1] != 0.0) {
                const double h = L / (p.n[d] + 1);
                const double s = std::sin(M_PI * h / (2.0 * L));
                mu += 4.0 / (h * h) * s * s;
            } else {
                mu += (M_PI / L) * (M_PI / L);
            }
        }
        r.ac_rate = -lam + p.kappa[0] * mu + p.q;
        r.ac_mu = mu;
        r.exp_lt = std::exp(-lam * t);
    }
    return r;
}

// Raise a kernel's dynamic-LDS limit once per instantiation (the attribute
// persists for the process).  `done` is the largest limit set so far; host
// threads that launch the same kernel at once may both set it, and it only
// grows.
template <typename K>
hipError_t set_lds(K kernel, size_t bytes, std::atomic<size_t>& done) {
    if (bytes <= done.load(std::memory_order_acquire)) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    if (e == hipSuccess) {
        size_t cur = done.load(std::memory_order_relaxed);
        while (cur < bytes && !done.compare_exchange_weak(cur, bytes, std::memory_order_release)) {
        }
    }
    return e;
}

// Tile shape of a stage launch.  Every wave owns `rb` 16-row blocks of each
// product (a tile has NP/(16 rb) waves) and a tile spans `cb` 16-column
// (outer stages) or 16-line (x stage) blocks, so that each P fragment read
// from L2 feeds 2*NC*cb MFMAs and each B fragment rb of them.  Instantiated
// (rb, cb, launch bound): (1,1,1024), (1,2,1024), (2,1,512), (2,1,1024),
// (4,1,1024), (2,2,512); with an FP32 state also (4,1,512) and (4,2,512),
// and for single-component x stages (2,4,512) and (1,4,1024).
//
// The default shape, measured on the 255^3 workload: for single-component
// FP64 systems up to NP = 256, one row block per wave over two column or line
// blocks (16 waves on one 132 KB tile: 2-5% faster than two row blocks per
// wave); otherwise rb = 2 up to NP = 512 and 4 beyond, two column blocks in
// the outer stages with an FP32 state, and x tiles of four line blocks for
// single-component FP32-state systems, two for other FP32 states (a
// two-component FP64 tile would spill).  An autotuned plan times every valid
// shape instead.
int shape_threads(int NP, int rb) { return 64 * (NP / (16 * rb)); }

template <typename T>
bool shape_rows_ok(int NP, int rb) {
    // eight row blocks per wave: FP32 state only (an FP64 tile would spill)
    if (rb != 1 && rb != 2 && rb != 4 && !(rb == 8 && sizeof(T) == 4)) return false;
    if (NP % (16 * rb) != 0 || NP / (16 * rb) > kMaxWaves) return false;
    return !(rb == 4 && shape_threads(NP, rb) <= 512 && sizeof(T) != 4);
}

template <typename T, int NC>
bool outer_shape_ok(int NP, TileShape t) {
    if (!shape_rows_ok<T>(NP, t.rb)) return false;
    if (t.cb == 2) {
        if (t.rb >= 2 && shape_threads(NP, t.rb) > 512) return false;
        if ((t.rb == 4 && sizeof(T) != 4) || t.rb == 8) return false;
    } else if (t.cb != 1) {
        return false;
    }
    return outer_lds_bytes(NP, 2 * NC, t.cb, sizeof(T)) <= kMaxLds;
}

template <typename T, int NC>
bool x_shape_ok(int NP, long nlines, TileShape t) {
    if (!shape_rows_ok<T>(NP, t.rb)) return false;
    // eight row blocks over two line blocks: the one-array tile of an FP32
    // state, for lines whose two-array two-block tile exceeds the LDS
    if (t.rb == 8 && t.cb == 2)
        return sizeof(T) == 4 && NC == 1 && nlines % 32 == 0 && x_lds_bytes(NP, 2, 2, sizeof(T)) > kMaxLds &&
               x_lds_bytes(NP, 1, 2, sizeof(T)) <= kMaxLds;
    if (t.cb == 2 || t.cb == 4) {
        if (t.rb >= 2 && shape_threads(NP, t.rb) > 512) return false;
        if ((t.rb == 4 && (t.cb == 4 || sizeof(T) != 4)) || t.rb == 8) return false;
        if (t.cb == 4 && !(sizeof(T) == 4 && NC == 1)) return false;
    } else if (t.cb != 1) {
        return false;
    }
    if (nlines % (16 * t.cb) != 0) return false;
    return x_lds_bytes(NP, 2 * NC, t.cb, sizeof(T)) <= kMaxLds;
}

template <typename T, int NC>
TileShape default_outer_shape(int NP) {
    if (sizeof(T) == 8 && NC == 1 && outer_shape_ok<T, NC>(NP, TileShape{1, 2})) return TileShape{1, 2};
    if (sizeof(T) == 4 && outer_shape_ok<T, NC>(NP, TileShape{2, 2})) return TileShape{2, 2};
    return TileShape{rows_per_wave(NP), 1};
}

template <typename T, int NC>
TileShape default_x_shape(int NP, long nlines) {
    if (sizeof(T) == 8 && NC == 1 && x_shape_ok<T, NC>(NP, nlines, TileShape{1, 2})) return TileShape{1, 2};
    if (sizeof(T) == 4 && NC == 1 && x_shape_ok<T, NC>(NP, nlines, TileShape{2, 4})) return TileShape{2, 4};
    if ((sizeof(T) == 4 || NC == 1) && x_shape_ok<T, NC>(NP, nlines, TileShape{2, 2})) return TileShape{2, 2};
    return TileShape{rows_per_wave(NP), 1};
}

// Defaults per matrix-core policy, measured on the 255^3 workload with the
// autotuner:
//  - split-BF16 products on an FP32 state take four row blocks per wave on
//    two column or line blocks (each split B fragment then feeds 24 MFMAs;
//    x stage 0.641 -> 0.570 ms per step against (2, 4));
//  - on an FP64 state, split-BF16 products take (2, 1) in every stage (1.068
//    -> 0.812 ms against the FP64 shapes) and FP32 products (2, 1) in the
//    outer stages and (2, 2) in the x stage (1.254 -> 1.166 ms).
template <typename M>
constexpr bool fp64_state_reduced() {
    return sizeof(typename M::elem) == 8 && sizeof(typename M::acc) == 4;
}

// A launch of at most kFewTiles one-block tiles leaves CUs idle with larger
// tiles, so it takes one row block per wave over one block (every tile shape
// gives the same result): at 63^2 FP64 the per-stage kernels take 11.4 (x)
// and 8.9 us (y) with two-block tiles on two CUs.  `copies`: instances that
// share the launch (a batch group).
constexpr long kFewTiles = 256;

template <typename M, int NC>
TileShape default_outer_for(int NP, long ncols16, long copies = 1) {
    typedef typename M::elem T;
    if (ncols16 * copies <= kFewTiles && outer_shape_ok<T, NC>(NP, TileShape{1, 1})) return TileShape{1, 1};
    if (fp64_state_reduced<M>() && outer_shape_ok<T, NC>(NP, TileShape{2, 1})) return TileShape{2, 1};
    if (M::SPLIT_B && NC == 1 && outer_shape_ok<T, NC>(NP, TileShape{4, 2})) return TileShape{4, 2};
    // FP32 products at NP = 256 with at least 1024 two-block tiles take four
    // row blocks as well (2.4% faster on the 255^3 workload; with few tiles,
    // as in one 2-D grid, the eight-wave (2, 2) tile keeps more waves busy)
    if (sizeof(T) == 4 && NC == 1 && NP == 256 && ncols16 >= 2048 && outer_shape_ok<T, NC>(NP, TileShape{4, 2}))
        return TileShape{4, 2};
    return default_outer_shape<T, NC>(NP);
}

template <typename M, int NC>
TileShape default_x_for(int NP, long nlines, long copies = 1) {
    typedef typename M::elem T;
    if (nlines / 16 * copies <= kFewTiles && x_shape_ok<T, NC>(NP, nlines, TileShape{1, 1})) return TileShape{1, 1};
    // lines too long for a two-array tile of two blocks: the one-array tile
    // (1024-point FP32 x stage 2.07 -> 1.48 ms against four row blocks over
    // one block; the 256-instance batch 16.7 -> 14.9 ms per step)
    if (!M::SPLIT_B && x_shape_ok<T, NC>(NP, nlines, TileShape{8, 2})) return TileShape{8, 2};
    // 512-point FP32 lines: four row blocks over two line blocks (x stage of a
    // 511 x 127^2 grid 0.51 -> 0.39 ms against two row blocks over one block
    // in 1024 threads; the 256-instance batch 15.1 -> 14.8 ms per step)
    if (sizeof(T) == 4 && !M::SPLIT_B && NC == 1 && NP == 512 && x_shape_ok<T, NC>(NP, nlines, TileShape{4, 2}))
        return TileShape{4, 2};
    // batch groups of FP32 lines with fewer than 1024 four-block tiles take two
    // line blocks: with so few large tiles the persistent launch ends on a
    // ragged last round (96 instances of 255^2: 0.364 -> 0.335 ms per step,
    // 48 of 127^2: 0.079 -> 0.067; single grids keep four, whose launches
    // measured faster: the x stage of 255 x 127^2 0.107 against 0.116 ms)
    if (sizeof(T) == 4 && !M::SPLIT_B && NC == 1 && copies > 1 && nlines / 64 * copies < 1024 &&
        x_shape_ok<T, NC>(NP, nlines, TileShape{2, 2}))
        return TileShape{2, 2};
    if (fp64_state_reduced<M>()) {
        if (!M::SPLIT_B && x_shape_ok<T, NC>(NP, nlines, TileShape{2, 2})) return TileShape{2, 2};
        if (x_shape_ok<T, NC>(NP, nlines, TileShape{2, 1})) return TileShape{2, 1};
    }
    if (M::SPLIT_B && sizeof(T) == 4 && NC == 1 && x_shape_ok<T, NC>(NP, nlines, TileShape{4, 2}))
        return TileShape{4, 2};
    return default_x_shape<T, NC>(NP, nlines);
}

int tile_threads(int NP) { return shape_threads(NP, rows_per_wave(NP)); }

// Launch kern<RB, MAXT> for the padded length NP with the default rows per
// wave: (2, 512) up to 256, (2, 1024) up to 512, (4, 1024) up to 1024.
#define DISPATCH_SHAPE(NP, KERNEL, ...)                                   \
    ((NP) <= 256 ? KERNEL(2, 512, __VA_ARGS__)                            \
                 : ((NP) <= 512 ? KERNEL(2, 1024, __VA_ARGS__) : KERNEL(4, 1024, __VA_ARGS__)))

// Workgroups of a kernel resident on the whole device at once (the grid of a
// persistent launch).  Each launcher caches it per instantiation and LDS size.
template <typename K>
long resident_groups(K kernel, int threads, size_t lds) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), threads, lds) !=
            hipSuccess ||
        per_cu < 1 || cus < 1)
        return 0;
    return long(per_cu) * cus;
}

struct GridCache {
    std::mutex m;
    size_t lds = 0;
    long resident = 0;
    // resident workgroups for `l` bytes of LDS (0 if the query failed)
    template <typename K>
    long resident_for(K kernel, int threads, size_t l) {
        std::lock_guard<std::mutex> lock(m);
        if (l != lds || resident == 0) {
            resident = resident_groups(kernel, threads, l);
            lds = l;
        }
        return resident;
    }
    template <typename K>
    long grid(K kernel, int threads, size_t l, long ntiles) {
        const long r = resident_for(kernel, threads, l);
        return r > 0 ? std::max(1L, std::min(ntiles, r)) : ntiles;
    }
};

template <typename M, int NC, bool FIRST, int RB, int CB, int MAXT>
etd_status launch_outer_k(const OuterArgs& a, long ntiles, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = outer_lds_bytes(a.NP, 2 * NC, CB, sizeof(T));
    auto k = outer_stage<M, NC, FIRST, RB, CB, MAXT>;
    static std::atomic<size_t> done{0};
    HIP_TRY(set_lds(k, lds, done), "outer stage LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(ntiles)), dim3(shape_threads(a.NP, RB)), lds, s, a);
    HIP_TRY(hipGetLastError(), "outer stage launch");
    return ETD_OK;
}

#define OUTER_K(RB, MAXT, M, NC, FIRST, CB, a, nb, s) launch_outer_k<M, NC, FIRST, RB, CB, MAXT>(a, nb, s)

template <typename M, int NC, bool FIRST, int RB, int CB, int MAXT>
etd_status launch_outer_group_k(const Group<OuterArgs>& g, int NP, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = outer_lds_bytes(NP, 2 * NC, CB, sizeof(T));
    auto k = outer_group<M, NC, FIRST, RB, CB, MAXT>;
    static std::atomic<size_t> done{0};
    static GridCache gc;
    HIP_TRY(set_lds(k, lds, done), "grouped outer stage LDS attribute");
    const int thr = shape_threads(NP, RB);
    hipLaunchKernelGGL(k, dim3(unsigned(gc.grid(k, thr, lds, g.ntiles))), dim3(thr), lds, s, g);
    HIP_TRY(hipGetLastError(), "grouped outer stage launch");
    return ETD_OK;
}

// Pick the instantiation of a valid shape: L is launch_outer_k or
// launch_outer_group_k applied through a generic lambda.
template <typename T, int NC, typename L>
etd_status outer_by_shape(int NP, TileShape t, L&& launch) {
    const bool small = shape_threads(NP, t.rb) <= 512;
    if (t.rb == 8) {
        if constexpr (sizeof(T) == 4)
            return launch(std::integral_constant<int, 8>{}, std::integral_constant<int, 1>{},
                          std::integral_constant<int, 512>{});
        return fail(ETD_EUNSUPPORTED, "tile shape not available at this precision");
    }
    if (t.rb == 1)
        return t.cb == 2 ? launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{},
                                  std::integral_constant<int, 1024>{})
                         : launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{},
                                  std::integral_constant<int, 1024>{});
    if (t.cb == 2) {
        if constexpr (sizeof(T) == 4)
            if (t.rb == 4)
                return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 2>{},
                              std::integral_constant<int, 512>{});
        return launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{},
                      std::integral_constant<int, 512>{});
    }
    if (t.rb == 2)
        return small ? launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{},
                              std::integral_constant<int, 512>{})
                     : launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{},
                              std::integral_constant<int, 1024>{});
    if (!small)
        return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{},
                      std::integral_constant<int, 1024>{});
    if constexpr (sizeof(T) == 4)
        return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{},
                      std::integral_constant<int, 512>{});
    return fail(ETD_EUNSUPPORTED, "tile shape not available at this precision");
}

// One outer stage over all components of one instance.  a.ncb and ncols16
// count 16-column blocks.  Systems whose joint tile exceeds the LDS run one
// component per launch with the default rows per wave.
template <typename M, int NC, bool FIRST>
etd_status launch_outer(OuterArgs a, long ncols16, TileShape t, hipStream_t s) {
    typedef typename M::elem T;
    if (NC == 2 && !outer_fused(a.NP, NC, sizeof(T))) {
        for (int c = 0; c < NC; ++c) {
            OuterArgs b = a;
            const long off = c * a.sc;
            b.in0 = static_cast<const T*>(a.in0) + off;
            b.in1 = FIRST ? nullptr : static_cast<const T*>(a.in1) + off;
            b.out0 = static_cast<T*>(a.out0) + off;
            b.out1 = static_cast<T*>(a.out1) + off;
            b.diag = static_cast<const T*>(a.diag) + c * a.diag_cstride;
            b.other = FIRST ? static_cast<const T*>(a.in0) + (1 - c) * a.sc : nullptr;
            b.comp = c;
            const etd_status st = DISPATCH_SHAPE(a.NP, OUTER_K, M, 1, FIRST, 1, b, ncols16, s);
            if (st != ETD_OK) return st;
        }
        return ETD_OK;
    }
    if (t.rb == 0) t = default_outer_for<M, NC>(a.NP, ncols16);
    a.ncb /= t.cb;
    return outer_by_shape<T, NC>(a.NP, t, [&](auto rb, auto cb, auto mt) {
        return launch_outer_k<M, NC, FIRST, decltype(rb)::value, decltype(cb)::value, decltype(mt)::value>(
            a, ncols16 / decltype(cb)::value, s);
    });
}

template <typename M, int NC, int RB, int CB, int MAXT>
etd_status launch_x_k(const XArgs& a, long nlines, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = x_lds_bytes(a.NP, x_one_array<M, NC, RB, CB>() ? 1 : 2 * NC, CB, sizeof(T));
    auto k = x_stage<M, NC, RB, CB, MAXT>;
    static std::atomic<size_t> done{0};
    HIP_TRY(set_lds(k, lds, done), "x stage LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(nlines / (16 * CB))), dim3(shape_threads(a.NP, RB)), lds, s, a);
    HIP_TRY(hipGetLastError(), "x stage launch");
    return ETD_OK;
}

template <typename M, int NC, int RB, int CB, int MAXT>
etd_status launch_x_group_k(const Group<XArgs>& g, int NP, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = x_lds_bytes(NP, x_one_array<M, NC, RB, CB>() ? 1 : 2 * NC, CB, sizeof(T));
    auto k = x_group<M, NC, RB, CB, MAXT>;
    static std::atomic<size_t> done{0};
    static GridCache gc;
    HIP_TRY(set_lds(k, lds, done), "grouped x stage LDS attribute");
    const int thr = shape_threads(NP, RB);
    hipLaunchKernelGGL(k, dim3(unsigned(gc.grid(k, thr, lds, g.ntiles))), dim3(thr), lds, s, g);
    HIP_TRY(hipGetLastError(), "grouped x stage launch");
    return ETD_OK;
}

template <typename T, int NC, typename L>
etd_status x_by_shape(int NP, TileShape t, L&& launch) {
    const bool small = shape_threads(NP, t.rb) <= 512;
    if (t.rb == 8) {
        if constexpr (sizeof(T) == 4) {
            if (t.cb == 2) {
                if constexpr (NC == 1)
                    return launch(std::integral_constant<int, 8>{}, std::integral_constant<int, 2>{},
                                  std::integral_constant<int, 512>{});
                return fail(ETD_EUNSUPPORTED, "tile shape not available for this system");
            }
            return launch(std::integral_constant<int, 8>{}, std::integral_constant<int, 1>{},
                          std::integral_constant<int, 512>{});
        }
        return fail(ETD_EUNSUPPORTED, "tile shape not available at this precision");
    }
    if (t.rb == 1) {
        if (t.cb == 4) {
            if constexpr (sizeof(T) == 4 && NC == 1)
                return launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 4>{},
                              std::integral_constant<int, 1024>{});
            return fail(ETD_EUNSUPPORTED, "tile shape not available for this system");
        }
        return t.cb == 2 ? launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{},
                                  std::integral_constant<int, 1024>{})
                         : launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{},
                                  std::integral_constant<int, 1024>{});
    }
    if (t.cb == 4) {
        if constexpr (sizeof(T) == 4 && NC == 1)
            return launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 4>{},
                          std::integral_constant<int, 512>{});
        return fail(ETD_EUNSUPPORTED, "tile shape not available for this system");
    }
    if (t.cb == 2) {
        if constexpr (sizeof(T) == 4)
            if (t.rb == 4)
                return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 2>{},
                              std::integral_constant<int, 512>{});
        return launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{},
                      std::integral_constant<int, 512>{});
    }
    if (t.rb == 2)
        return small ? launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{},
                              std::integral_constant<int, 512>{})
                     : launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{},
                              std::integral_constant<int, 1024>{});
    if (!small)
        return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{},
                      std::integral_constant<int, 1024>{});
    if constexpr (sizeof(T) == 4)
        return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{},
                      std::integral_constant<int, 512>{});
    return fail(ETD_EUNSUPPORTED, "tile shape not available at this precision");
}

template <typename M, int RB, int MAXT, bool SECOND>
etd_status launch_xsplit_k(const XSplitArgs& a, long nlines, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = x_lds_bytes(a.NP, 2, 1, sizeof(T));
    auto k = SECOND ? x_stage_u<M, RB, MAXT> : x_stage_w<M, RB, MAXT>;
    static std::atomic<size_t> done{0};
    HIP_TRY(set_lds(k, lds, done), "split x stage LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(nlines / 16)), dim3(tile_threads(a.NP)), lds, s, a);
    HIP_TRY(hipGetLastError(), "split x stage launch");
    return ETD_OK;
}

#define XS_K(RB, MAXT, M, SECOND, a, nl, s) launch_xsplit_k<M, RB, MAXT, SECOND>(a, nl, s)

// The x stage over all components of one instance.  `scratch` receives W
// when a system is split (its joint tile exceeds the LDS).
template <typename M, int NC>
etd_status launch_x(const XArgs& a, long nlines, TileShape t, typename M::elem* scratch, hipStream_t s) {
    typedef typename M::elem T;
    if (NC == 2 && !x_fused(a.NP, NC, sizeof(T))) {
        XSplitArgs b{};
        b.P = a.P;
        b.diag_sstride = a.diag_sstride;
        b.NP = a.NP;
        b.sc = a.sc;
        b.npy = a.npy;
        b.tau = a.tau;
        b.rxn = a.rxn;
        b.W = scratch;
        for (int c = 0; c < NC; ++c) {
            b.w3 = static_cast<const T*>(a.w3) + c * a.sc;
            b.w4 = static_cast<const T*>(a.w4) + c * a.sc;
            b.out = scratch + c * a.sc;
            b.diag = static_cast<const T*>(a.diag) + c * a.diag_cstride;
            b.comp = c;
            const etd_status st = DISPATCH_SHAPE(a.NP, XS_K, M, false, b, nlines, s);
            if (st != ETD_OK) return st;
        }
        for (int c = 0; c < NC; ++c) {
            b.w4 = static_cast<const T*>(a.w4) + c * a.sc;
            b.out = static_cast<T*>(a.out) + c * a.sc;
            b.diag = static_cast<const T*>(a.diag) + c * a.diag_cstride;
            b.comp = c;
            const etd_status st = DISPATCH_SHAPE(a.NP, XS_K, M, true, b, nlines, s);
            if (st != ETD_OK) return st;
        }
        return ETD_OK;
    }
    if (t.rb == 0) t = default_x_for<M, NC>(a.NP, nlines);
    return x_by_shape<T, NC>(a.NP, t, [&](auto rb, auto cb, auto mt) {
        return launch_x_k<M, NC, decltype(rb)::value, decltype(cb)::value, decltype(mt)::value>(a, nlines, s);
    });
}

TileShape plan_tile(const Plan& pl, int d) { return TileShape{pl.tile_rb[d], pl.tile_cb[d]}; }

etd_status timer_mark(StageTimer& t, int kind, bool begin, hipStream_t s);

#define TIMED(kind, call)                                           \
    do {                                                            \
        etd_status st_ = timer_mark(tm, kind, true, s);             \
        if (st_ != ETD_OK) return st_;                              \
        st_ = (call);                                               \
        if (st_ != ETD_OK) return st_;                              \
        st_ = timer_mark(tm, kind, false, s);                       \
        if (st_ != ETD_OK) return st_;                              \
    } while (0)

// Arguments of one step's stage launches for one instance whose workspace
// region starts at ws (times are filled in per step).  Pdir[d] is the P table
// the instance uses for direction d (a batch shares one per extent).
// outer[k] / ocols[k]: the k-th outer stage and its 16-column blocks;
// nlines: x lines.  Default tile shapes are applied by the launchers.
struct StepArgs {
    int nouter = 0;
    OuterArgs outer[2];
    long ocols[2] = {0, 0};
    int odir[2] = {0, 0};   // contracted direction of each outer stage
    XArgs x;
    long nlines = 0;
    void* split_scratch = nullptr;   // W of a split x stage
};

StepArgs step_args(const Plan& pl, char* ws, const void* const Pdir[3]) {
    const int px = pl.np[0], py = pl.np[1], pz = pl.np[2];
    const long sc = long(px) * py * pz;
    const size_t e = pl.elem;
    char* U = ws + pl.lay.field[0];
    char* WA = ws + pl.lay.field[1];
    char* WB = ws + pl.lay.field[2];
    char* WC = ws + pl.lay.field[3];
    char* WD = ws + pl.lay.field[4];
    const char* diag = ws + pl.lay.diag;
    const long dstride = long(pl.diag_stride);
    const long dcs = long(kDiagSlots) * dstride;
    StepArgs a;
    OuterArgs o{};
    o.diag_cstride = dcs;
    o.sc = sc;
    o.npx = px;
    o.npy = py;
    o.dim = pl.dim;
    const char* w3;
    const char* w4;
    if (pl.dim == 3) {
        // z stage: contracted index z (stride px*py), columns (y, x)
        o.in0 = U;
        o.in1 = nullptr;
        o.out0 = WA;
        o.out1 = WB;
        o.P = Pdir[2];
        o.diag = diag + long(kDiagZ) * dstride * e;
        o.NP = pz;
        o.ncb = px * py / 16;
        o.sk = long(px) * py;
        o.sb = 0;
        a.outer[0] = o;
        a.ocols[0] = o.ncb;
        a.odir[0] = 2;
        // y stage: contracted index y (stride px), columns x, batches z
        o.in0 = WA;
        o.in1 = WB;
        o.out0 = WC;
        o.out1 = WD;
        o.P = Pdir[1];
        o.diag = diag + long(kDiagY) * dstride * e;
        o.NP = py;
        o.ncb = px / 16;
        o.sk = px;
        o.sb = long(px) * py;
        a.outer[1] = o;
        a.ocols[1] = long(o.ncb) * pz;
        a.odir[1] = 1;
        a.nouter = 2;
        w3 = WC;
        w4 = WD;
        a.split_scratch = WA;
    } else {
        o.in0 = U;
        o.in1 = nullptr;
        o.out0 = WA;
        o.out1 = WB;
        o.P = Pdir[1];
        o.diag = diag + long(kDiagY) * dstride * e;
        o.NP = py;
        o.ncb = px / 16;
        o.sk = px;
        o.sb = 0;
        a.outer[0] = o;
        a.ocols[0] = o.ncb;
        a.odir[0] = 1;
        a.nouter = 1;
        w3 = WA;
        w4 = WB;
        a.split_scratch = WC;
    }
    XArgs& x = a.x;
    x = XArgs{};
    x.w3 = w3;
    x.w4 = w4;
    x.out = U;
    x.P = Pdir[0];
    x.diag = diag + long(kDiagX1) * dstride * e;
    x.diag_sstride = dstride;
    x.diag_cstride = dcs;
    x.NP = px;
    x.sc = sc;
    x.npy = py;
    x.tau = pl.prob.tau;
    x.Wout = nullptr;
    a.nlines = long(py) * pz;
    return a;
}

// One product-parallel launch: row groups of 16*NW rows x 16-column tiles,
// as a one-dimensional grid (split_block maps it XCD by XCD).
template <typename M, int NC, int KIND, int NW, int BK, int KS>
etd_status launch_split_k(const SplitArgs& a, long ncols, hipStream_t s) {
    typedef typename M::elem T;
    if (a.NP % (BK * KS) != 0) return fail(ETD_EINVAL, "2-D product chunks do not divide the padded extent");
    const size_t lds = split_lds_bytes(SplitShape<KIND, NC>::NARR, BK, KS, sizeof(T));
    auto k = split_product<M, NC, KIND, NW, BK, KS>;
    static std::atomic<size_t> done{0};
    HIP_TRY(set_lds(k, lds, done), "2-D product LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(a.NP / (16 * NW) * (ncols / 16))), dim3(64 * NW * KS), lds, s, a);
    HIP_TRY(hipGetLastError(), "2-D product launch");
    return ETD_OK;
}

// Chunks and contraction parts: an FP64 state takes four parts of 32-index
// chunks (four waves per SIMD; 511^2 two-component FP64 step 0.137 -> 0.131
// ms against two parts of 64), an FP32 state two parts of 128-index chunks
// (four parts: 0.081 -> 0.083 ms); smaller chunks and fewer parts where the
// padded extent (a multiple of 32) is not divisible.
template <typename M, int NC, int KIND, int NW>
etd_status launch_split_bk(const SplitArgs& a, long ncols, hipStream_t s) {
    typedef typename M::elem T;
    if constexpr (sizeof(T) == 4) {
        if (a.NP % 256 == 0) return launch_split_k<M, NC, KIND, NW, 128, 2>(a, ncols, s);
    } else {
        if (a.NP % 128 == 0) return launch_split_k<M, NC, KIND, NW, 32, 4>(a, ncols, s);
    }
    if (a.NP % 128 == 0) return launch_split_k<M, NC, KIND, NW, 64, 2>(a, ncols, s);
    if (a.NP % 64 == 0) return launch_split_k<M, NC, KIND, NW, 32, 2>(a, ncols, s);
    return launch_split_k<M, NC, KIND, NW, 32, 1>(a, ncols, s);
}

template <typename M, int NC, int KIND>
etd_status launch_split(const SplitArgs& a, long ncols, hipStream_t s) {
    return a.NP % 64 == 0 ? launch_split_bk<M, NC, KIND, 4>(a, ncols, s) : launch_split_bk<M, NC, KIND, 2>(a, ncols, s);
}

// 2-D problems take the product-parallel path when it has at least 128
// blocks per launch (NP_y / 64 row groups x NP_x / 16 column tiles; from
// about 512^2 on), where the fused stages would have only NP_x / 16 tiles.
bool use_split2d(const Plan& pl) { return pl.dim == 2 && long(pl.np[1] / 64) * (pl.np[0] / 16) >= 128; }

template <typename M, int NC>
etd_status run_steps_split2d(const Plan& pl, StageTimer& tm, char* ws, double t0, int nsteps, hipStream_t s) {
    typedef typename M::elem T;
    const long dstride = long(pl.diag_stride);
    const char* diag = ws + pl.lay.diag;
    SplitArgs a{};
    a.U = ws + pl.lay.field[0];
    a.WA = ws + pl.lay.field[1];
    a.WB = ws + pl.lay.field[2];
    a.WC = ws + pl.lay.field[3];
    a.WD = ws + pl.lay.field[4];
    a.diag_sstride = dstride;
    a.diag_cstride = long(kDiagSlots) * dstride;
    a.npx = pl.np[0];
    a.sc = long(pl.np[0]) * pl.np[1];
    a.tau = pl.prob.tau;
    SplitArgs y = a, x = a;
    y.P = ws + pl.lay.P[1];
    y.diag = diag + long(kDiagY) * dstride * pl.elem;
    y.NP = pl.np[1];
    x.P = ws + pl.lay.P[0];
    x.diag = diag + long(kDiagX1) * dstride * pl.elem;
    x.NP = pl.np[0];
    const long nx = pl.np[0], ny = pl.np[1];
    for (int step = 0; step < nsteps; ++step) {
        y.rxn = rxn_args(pl, ws, t0 + step * pl.prob.tau);
        x.rxn = rxn_args(pl, ws, t0 + (step + 1) * pl.prob.tau);
        TIMED(0, (launch_split<M, NC, kSplitYF>(y, nx, s)));
        TIMED(0, (launch_split<M, NC, kSplitYB>(y, nx, s)));
        TIMED(2, (launch_split<M, NC, kSplitX1>(x, ny, s)));
        TIMED(2, (launch_split<M, NC, kSplitX2>(x, ny, s)));
        TIMED(2, (launch_split<M, NC, kSplitX3>(x, ny, s)));
        TIMED(2, (launch_split<M, NC, kSplitX4>(x, ny, s)));
    }
    return ETD_OK;
}

// Resident schedule (ETD_SCHEDULE_RESIDENT): every step of a run in one
// cooperative launch, for grids whose directions share one padded extent of at
// most kResidentMaxNP points (fused tiles of one row block per wave and one
// column or line block: NP/16 waves).  AUTO does not take it: with one-block
// tiles the per-stage launches are as fast on small grids (63^2 FP64, 100-step
// calls: 15.2 us per step against 14.9 resident; 127^2: 32.8 against 35.1;
// a graph of per-stage launches 14.3 us at 63^2), a cooperative launch costs
// 40-180 us of host time, and the grid-wide barrier's cost grows with the
// workgroup count (63^3: 25 against 105 us).
constexpr int kResidentMaxNP = 128;
constexpr int kResidentThreads = 512;

bool resident_eligible(const Plan& pl) {
    const int NP = pl.np[0];
    if (NP > kResidentMaxNP) return false;
    for (int d = 1; d < pl.dim; ++d)
        if (pl.np[d] != NP) return false;
    return !use_split2d(pl);
}

bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus c = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &c) == hipSuccess && c != hipStreamCaptureStatusNone;
}

// The schedule a run takes: ETD_SCHEDULE_STAGES or ETD_SCHEDULE_RESIDENT, or
// ETD_SCHEDULE_AUTO if a forced resident schedule cannot run here (capture).
int resolve_schedule(const Plan& pl, hipStream_t s) {
    if (pl.schedule != ETD_SCHEDULE_RESIDENT || !resident_eligible(pl)) return ETD_SCHEDULE_STAGES;
    return stream_capturing(s) ? ETD_SCHEDULE_AUTO : ETD_SCHEDULE_RESIDENT;
}

template <typename M, int NC>
etd_status run_steps_resident(const Plan& pl, char* ws, double t0, int nsteps, hipStream_t s) {
    typedef typename M::elem T;
    const void* Pdir[3] = {ws + pl.lay.P[0], ws + pl.lay.P[1], ws + pl.lay.P[2]};
    const StepArgs st = step_args(pl, ws, Pdir);
    ResidentArgs a{};
    a.nouter = st.nouter;
    long ntiles = st.nlines / 16;
    for (int k = 0; k < st.nouter; ++k) {
        a.outer[k] = st.outer[k];
        a.outer[k].rxn = rxn_args(pl, ws, t0);   // the kernel sets each step's time
        a.otiles[k] = st.ocols[k];
        ntiles = std::max(ntiles, a.otiles[k]);
    }
    a.x = st.x;
    a.x.rxn = rxn_args(pl, ws, t0);
    a.xtiles = st.nlines / 16;
    a.nsteps = nsteps;
    a.t0 = t0;
    const int NP = pl.np[0];
    const size_t lds = std::max(outer_lds_bytes(NP, 2 * NC, 1, sizeof(T)), x_lds_bytes(NP, 2 * NC, 1, sizeof(T)));
    const int thr = shape_threads(NP, 1);
    auto k = resident_steps<M, NC, kResidentThreads>;
    static std::atomic<size_t> done{0};
    static GridCache gc;
    static std::atomic<int> coop{-1};
    if (coop.load() < 0) {
        int dev = 0, c = 0;
        HIP_TRY(hipGetDevice(&dev), "device query");
        HIP_TRY(hipDeviceGetAttribute(&c, hipDeviceAttributeCooperativeLaunch, dev), "cooperative launch query");
        coop.store(c);
    }
    if (!coop.load()) return fail(ETD_EUNSUPPORTED, "the device does not support cooperative launches");
    HIP_TRY(set_lds(k, lds, done), "resident schedule LDS attribute");
    const long cap = gc.resident_for(k, thr, lds);
    if (cap < 1) return fail(ETD_EHIP, "resident schedule: occupancy query failed");
    const long grid = std::max(1L, std::min(ntiles, cap));
    void* args[] = {&a};
    HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k), dim3(unsigned(grid)), dim3(thr), args,
                                       unsigned(lds), s),
            "resident schedule launch");
    return ETD_OK;
}

template <typename M, int NC>
etd_status run_steps(const Plan& pl, StageTimer& tm, char* ws, double t0, int nsteps, hipStream_t s,
                     typename M::elem* w_out = nullptr) {
    typedef typename M::elem T;
    if (w_out == nullptr && use_split2d(pl)) return run_steps_split2d<M, NC>(pl, tm, ws, t0, nsteps, s);
    if (w_out == nullptr) {
        const int sch = resolve_schedule(pl, s);
        if (sch == ETD_SCHEDULE_AUTO)
            return fail(ETD_EUNSUPPORTED, "the resident schedule is one cooperative launch and cannot be captured");
        if (sch == ETD_SCHEDULE_RESIDENT) return run_steps_resident<M, NC>(pl, ws, t0, nsteps, s);
    }
    const void* Pdir[3] = {ws + pl.lay.P[0], ws + pl.lay.P[1], ws + pl.lay.P[2]};
    StepArgs a = step_args(pl, ws, Pdir);
    a.x.Wout = w_out;
    const double tau = pl.prob.tau;
    for (int step = 0; step < nsteps; ++step) {
        const double tn = t0 + step * tau;
        const double tn1 = t0 + (step + 1) * tau;
        for (int k = 0; k < a.nouter; ++k) {
            a.outer[k].rxn = rxn_args(pl, ws, tn);
            if (k == 0) TIMED(0, (launch_outer<M, NC, true>(a.outer[0], a.ocols[0], plan_tile(pl, a.odir[0]), s)));
            else TIMED(1, (launch_outer<M, NC, false>(a.outer[1], a.ocols[1], plan_tile(pl, a.odir[1]), s)));
        }
        a.x.rxn = rxn_args(pl, ws, tn1);
        TIMED(2, (launch_x<M, NC>(a.x, a.nlines, plan_tile(pl, 0), static_cast<T*>(a.split_scratch), s)));
    }
    return ETD_OK;
}

// One step from Uin to Uout (padded fields, any buffers) that keeps its stage
// fields: f = [w1, w2, w3, w4, W] in 3-D, [w1, w2, W] in 2-D (w1, w2 the
// first stage's outputs, W the x stage's).  Fused tiles only (the adjoint's
// own limits imply them).
template <typename M, int NC>
etd_status replay_step(const Plan& pl, StageTimer& tm, char* ws, double tn, const void* Uin, void* Uout,
                       char* const* f, hipStream_t s) {
    typedef typename M::elem T;
    const void* Pdir[3] = {ws + pl.lay.P[0], ws + pl.lay.P[1], ws + pl.lay.P[2]};
    StepArgs a = step_args(pl, ws, Pdir);
    a.outer[0].in0 = Uin;
    a.outer[0].out0 = f[0];
    a.outer[0].out1 = f[1];
    if (pl.dim == 3) {
        a.outer[1].in0 = f[0];
        a.outer[1].in1 = f[1];
        a.outer[1].out0 = f[2];
        a.outer[1].out1 = f[3];
        a.x.w3 = f[2];
        a.x.w4 = f[3];
        a.x.Wout = f[4];
    } else {
        a.x.w3 = f[0];
        a.x.w4 = f[1];
        a.x.Wout = f[2];
    }
    a.x.out = Uout;
    for (int k = 0; k < a.nouter; ++k) {
        a.outer[k].rxn = rxn_args(pl, ws, tn);
        if (k == 0) TIMED(0, (launch_outer<M, NC, true>(a.outer[0], a.ocols[0], plan_tile(pl, a.odir[0]), s)));
        else TIMED(1, (launch_outer<M, NC, false>(a.outer[1], a.ocols[1], plan_tile(pl, a.odir[1]), s)));
    }
    a.x.rxn = rxn_args(pl, ws, tn + pl.prob.tau);
    TIMED(2, (launch_x<M, NC>(a.x, a.nlines, plan_tile(pl, 0), reinterpret_cast<T*>(ws + pl.lay.field[4]), s)));
    return ETD_OK;
}

template <typename M>
etd_status advance_m(const Plan& pl, StageTimer& tm, void* u, double t0, int nsteps, char* ws, hipStream_t s) {
    typedef typename M::elem T;
    const Dims d = dims_of(pl);
    T* U = reinterpret_cast<T*>(ws + pl.lay.field[0]);
    hipLaunchKernelGGL(pack_field<T>, dim3(2048), dim3(256), 0, s, static_cast<const T*>(u), U, d);
    HIP_TRY(hipGetLastError(), "pack launch");
    etd_status st = pl.nc == 1 ? run_steps<M, 1>(pl, tm, ws, t0, nsteps, s) : run_steps<M, 2>(pl, tm, ws, t0, nsteps, s);
    if (st != ETD_OK) return st;
    hipLaunchKernelGGL(unpack_field<T>, dim3(2048), dim3(256), 0, s, U, static_cast<T*>(u), d);
    HIP_TRY(hipGetLastError(), "unpack launch");
    return ETD_OK;
}

}  // namespace
