// Tile-shape autotuning.
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

// ---------------------------------------------------------------------------
// Autotuning: time every valid tile shape of a stage and keep the fastest.
// All shapes compute every output with the same operations in the same
// order, so the choice changes the speed, never the result.
// ---------------------------------------------------------------------------

template <typename T, int NC>
std::vector<TileShape> outer_candidates(int NP) {
    std::vector<TileShape> v;
    for (int rb : {1, 2, 4, 8})
        for (int cb : {1, 2})
            if (outer_shape_ok<T, NC>(NP, TileShape{rb, cb})) v.push_back(TileShape{rb, cb});
    return v;
}

template <typename T, int NC>
std::vector<TileShape> x_candidates(int NP, long nlines) {
    std::vector<TileShape> v;
    for (int rb : {1, 2, 4, 8})
        for (int cb : {1, 2, 4})
            if (x_shape_ok<T, NC>(NP, nlines, TileShape{rb, cb})) v.push_back(TileShape{rb, cb});
    return v;
}

// Mean milliseconds of `launch` over `reps` launches after one warm-up.
template <typename L>
etd_status time_launches(L&& launch, int reps, hipStream_t s, float& ms) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "autotune event");
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "autotune event");
    }
    etd_status st = launch();
    if (st == ETD_OK) {
        he = hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == ETD_OK; ++r) st = launch();
        if (he == hipSuccess) he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (st == ETD_OK && he != hipSuccess) st = hip_fail(he, "autotune timing");
        ms /= float(reps);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

constexpr int kTuneReps = 5;
constexpr int kMaxBatch = 4096;   // instances per batch

template <typename M, int NC>
etd_status autotune_plan_t(Plan& pl, char* ws, hipStream_t s) {
    typedef typename M::elem T;
    if (NC == 2 && (!x_fused(pl.np[0], NC, sizeof(T)) ||
                    !outer_fused(pl.np[1], NC, sizeof(T)) || (pl.dim == 3 && !outer_fused(pl.np[2], NC, sizeof(T)))))
        return ETD_OK;   // split systems run one fixed shape
    const void* Pdir[3] = {ws + pl.lay.P[0], ws + pl.lay.P[1], ws + pl.lay.P[2]};
    StepArgs a = step_args(pl, ws, Pdir);
    for (int k = 0; k < a.nouter; ++k) a.outer[k].rxn = rxn_args(pl, ws, 0.0);
    a.x.rxn = rxn_args(pl, ws, pl.prob.tau);
    for (int k = 0; k < a.nouter; ++k) {
        const int d = a.odir[k];
        TileShape best{};
        float best_ms = 0.f;
        for (TileShape t : outer_candidates<T, NC>(pl.np[d])) {
            float ms = 0.f;
            const etd_status st = time_launches([&]() {
                return k == 0 ? launch_outer<M, NC, true>(a.outer[0], a.ocols[0], t, s)
                              : launch_outer<M, NC, false>(a.outer[1], a.ocols[1], t, s);
            }, kTuneReps, s, ms);
            if (st != ETD_OK) return st;
            if (best.rb == 0 || ms < best_ms) {
                best = t;
                best_ms = ms;
            }
        }
        pl.tile_rb[d] = best.rb;
        pl.tile_cb[d] = best.cb;
    }
    TileShape best{};
    float best_ms = 0.f;
    for (TileShape t : x_candidates<T, NC>(pl.np[0], a.nlines)) {
        float ms = 0.f;
        const etd_status st = time_launches(
            [&]() { return launch_x<M, NC>(a.x, a.nlines, t, static_cast<T*>(a.split_scratch), s); }, kTuneReps, s,
            ms);
        if (st != ETD_OK) return st;
        if (best.rb == 0 || ms < best_ms) {
            best = t;
            best_ms = ms;
        }
    }
    pl.tile_rb[0] = best.rb;
    pl.tile_cb[0] = best.cb;
    return ETD_OK;
}

// Validate and resolve a tile request for one direction of a plan: (0, 0)
// selects the default shape (`copies`: instances sharing each launch).
template <typename M, int NC>
etd_status resolve_tile(const Plan& pl, int d, TileShape t, TileShape& out, long copies) {
    typedef typename M::elem T;
    const int NP = pl.np[d];
    const long nlines = long(pl.np[1]) * pl.np[2];
    if (t.rb == 0 && t.cb == 0) {
        const long ncols16 = long(pl.np[0]) * pl.np[1] * pl.np[2] / NP / 16;
        out = d == 0 ? default_x_for<M, NC>(NP, nlines, copies) : default_outer_for<M, NC>(NP, ncols16, copies);
        return ETD_OK;
    }
    const bool ok = d == 0 ? x_shape_ok<T, NC>(NP, nlines, t) : outer_shape_ok<T, NC>(NP, t);
    if (!ok) return fail(ETD_EUNSUPPORTED, "tile shape not valid for this direction");
    out = t;
    return ETD_OK;
}

}  // namespace
