// Batches of independent instances (grouped persistent launches).
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

// ---------------------------------------------------------------------------
// Batches: many independent instances (same dimension, component count and
// precision; any extents, coefficients, step, reaction and Pade order)
// advanced together.  Instances of one padded shape form a group; each group
// runs every stage of every step as ONE persistent grouped launch over all of
// its instances' tiles, on a stream of its own, so groups of different shapes
// overlap on the device.  Instances of equal extent share one P table.
// ---------------------------------------------------------------------------

size_t desc_bytes_of(const Batch& B) {
    size_t n = 0;
    for (const BatchGroup& G : B.groups) {
        const size_t k = G.inst.size();
        n += size_t(B.dim - 1) * a256(k * sizeof(OuterArgs)) + size_t(B.dim - 1) * a256((k + 1) * sizeof(long));
        n += a256(k * sizeof(XArgs)) + a256((k + 1) * sizeof(long));
    }
    return n;
}

etd_status batch_layout(Batch& B) {
    for (int d = 0; d < 3; ++d) {
        B.powner[d].assign(B.plans.size(), 0);
        for (size_t i = 0; i < B.plans.size(); ++i) {
            size_t j = 0;
            while (j < i && !(B.plans[j].n[d] == B.plans[i].n[d] && B.plans[j].np[d] == B.plans[i].np[d])) ++j;
            B.powner[d][i] = int(j);
        }
    }
    // The P tables lead a plan's layout.  An instance that takes every
    // direction's P from an earlier instance holds none of them: its region
    // starts at its first table after P, and its (unused) P offsets fall on
    // earlier regions, which it never reads or writes.  The owner of an
    // extent comes first and keeps its whole region, so the base stays >= 0.
    size_t off = 0;
    B.base.resize(B.plans.size());
    B.skip.assign(B.plans.size(), 0);
    for (size_t i = 0; i < B.plans.size(); ++i) {
        const Plan& pl = B.plans[i];
        bool borrows_all = true;
        for (int d = 0; d < pl.dim; ++d) borrows_all = borrows_all && B.powner[d][i] != int(i);
        // (earlier regions hold the owners' P of the same sizes, so off >=
        // pl.lay.diag whenever every direction is borrowed; kept as a check)
        const size_t skip = borrows_all && off >= pl.lay.diag ? pl.lay.diag : 0;
        B.skip[i] = skip;
        B.base[i] = off - skip;
        off = a256(off + pl.lay.total - skip);
    }
    for (size_t i = 0; i < B.plans.size(); ++i) {
        const Plan& pl = B.plans[i];
        size_t g = 0;
        while (g < B.groups.size() &&
               !(B.groups[g].np[0] == pl.np[0] && B.groups[g].np[1] == pl.np[1] && B.groups[g].np[2] == pl.np[2]))
            ++g;
        if (g == B.groups.size()) {
            BatchGroup G;
            for (int d = 0; d < 3; ++d) G.np[d] = pl.np[d];
            B.groups.push_back(G);
        }
        B.groups[g].inst.push_back(int(i));
    }
    B.desc = off;
    B.desc_bytes = desc_bytes_of(B);
    B.total = a256(off + B.desc_bytes);
    return ETD_OK;
}

// Host image of one group's descriptors for the workspace at ws, with the
// group's current tile shapes.
void group_descriptors(const Batch& B, BatchGroup& G, char* ws, size_t& off, std::vector<uint8_t>& img) {
    const int k = int(G.inst.size());
    std::vector<OuterArgs> oa[2];
    std::vector<long> os[2];
    std::vector<XArgs> xa;
    std::vector<long> xs;
    for (int j = 0; j < 2; ++j) os[j].push_back(0);
    xs.push_back(0);
    for (int i : G.inst) {
        const Plan& pl = B.plans[i];
        const void* Pdir[3];
        for (int d = 0; d < 3; ++d) {
            const int o = B.powner[d][i];
            Pdir[d] = ws + B.base[o] + B.plans[o].lay.P[d];
        }
        StepArgs a = step_args(pl, ws + B.base[i], Pdir);
        for (int j = 0; j < a.nouter; ++j) {
            const TileShape t = G.tile[a.odir[j]];
            a.outer[j].rxn = rxn_args(pl, ws + B.base[i], 0.0);
            a.outer[j].ncb /= t.cb;
            oa[j].push_back(a.outer[j]);
            os[j].push_back(os[j].back() + a.ocols[j] / t.cb);
        }
        a.x.rxn = rxn_args(pl, ws + B.base[i], 0.0);
        xa.push_back(a.x);
        xs.push_back(xs.back() + a.nlines / (16 * G.tile[0].cb));
    }
    auto put_bytes = [&](const void* src, size_t n) {
        const size_t at = off;
        std::memcpy(img.data() + (at - B.desc), src, n);
        off = a256(off + n);
        return at;
    };
    for (int j = 0; j < B.dim - 1; ++j) {
        G.oargs[j] = put_bytes(oa[j].data(), k * sizeof(OuterArgs));
        G.ostart[j] = put_bytes(os[j].data(), (k + 1) * sizeof(long));
        G.otiles[j] = os[j].back();
    }
    G.xargs = put_bytes(xa.data(), k * sizeof(XArgs));
    G.xstart = put_bytes(xs.data(), (k + 1) * sizeof(long));
    G.xtiles = xs.back();
}

// Rebuild and upload every group's descriptors (synchronous on s).
etd_status upload_descriptors(Batch& B, char* ws, hipStream_t s) {
    std::vector<uint8_t> img(B.desc_bytes, 0);
    size_t off = B.desc;
    for (BatchGroup& G : B.groups) group_descriptors(B, G, ws, off, img);
    HIP_TRY(hipMemcpyAsync(ws + B.desc, img.data(), img.size(), hipMemcpyHostToDevice, s), "descriptor upload");
    HIP_TRY(hipStreamSynchronize(s), "descriptor upload sync");
    B.uploaded = ws;
    ++*B.generation;
    return ETD_OK;
}

// One stage of one step for every instance of a group: stage 0 = first outer
// stage, 1 = middle outer stage (3-D), 2 = x stage.
template <typename M, int NC>
etd_status group_stage(const Batch& B, const BatchGroup& G, int stage, char* ws, double t0, int k, hipStream_t s) {
    typedef typename M::elem T;
    const int n = int(G.inst.size());
    if (stage < 2) {
        const int d = B.dim == 3 ? (stage == 0 ? 2 : 1) : 1;
        const int NP = G.np[d];
        Group<OuterArgs> g{reinterpret_cast<const OuterArgs*>(ws + G.oargs[stage]),
                           reinterpret_cast<const long*>(ws + G.ostart[stage]), n, G.otiles[stage], t0, k};
        if (stage == 0)
            return outer_by_shape<T, NC>(NP, G.tile[d], [&](auto rb, auto cb, auto mt) {
                return launch_outer_group_k<M, NC, true, decltype(rb)::value, decltype(cb)::value,
                                            decltype(mt)::value>(g, NP, s);
            });
        return outer_by_shape<T, NC>(NP, G.tile[d], [&](auto rb, auto cb, auto mt) {
            return launch_outer_group_k<M, NC, false, decltype(rb)::value, decltype(cb)::value, decltype(mt)::value>(
                g, NP, s);
        });
    }
    Group<XArgs> g{reinterpret_cast<const XArgs*>(ws + G.xargs), reinterpret_cast<const long*>(ws + G.xstart), n,
                   G.xtiles, t0, k};
    return x_by_shape<T, NC>(G.np[0], G.tile[0], [&](auto rb, auto cb, auto mt) {
        return launch_x_group_k<M, NC, decltype(rb)::value, decltype(cb)::value, decltype(mt)::value>(g, G.np[0], s);
    });
}

template <typename M, int NC>
etd_status batch_advance_t(Batch& B, void* const* u, double t0, int nsteps, char* ws, hipStream_t s) {
    typedef typename M::elem T;
    const bool fork = B.groups.size() > 1;
    if (fork) HIP_TRY(hipEventRecord(B.fork, s), "batch fork record");
    etd_status st = ETD_OK;
    for (BatchGroup& G : B.groups) {
        hipStream_t gs = fork ? G.stream : s;
        if (fork) {
            const hipError_t e = hipStreamWaitEvent(gs, B.fork, 0);
            if (e != hipSuccess) return hip_fail(e, "batch fork wait");
        }
        // the group's work; on an error the group is still joined below
        st = [&]() -> etd_status {
            for (int i : G.inst) {
                const Plan& pl = B.plans[i];
                hipLaunchKernelGGL(pack_field<T>, dim3(1024), dim3(256), 0, gs, static_cast<const T*>(u[i]),
                                   reinterpret_cast<T*>(ws + B.base[i] + pl.lay.field[0]), dims_of(pl));
            }
            HIP_TRY(hipGetLastError(), "batch pack launch");
            for (int step = 0; step < nsteps; ++step) {
                for (int stage = 0; stage < B.dim - 1; ++stage)
                    TRY((group_stage<M, NC>(B, G, stage, ws, t0, step, gs)));
                TRY((group_stage<M, NC>(B, G, 2, ws, t0, step + 1, gs)));
            }
            for (int i : G.inst) {
                const Plan& pl = B.plans[i];
                hipLaunchKernelGGL(unpack_field<T>, dim3(1024), dim3(256), 0, gs,
                                   reinterpret_cast<const T*>(ws + B.base[i] + pl.lay.field[0]),
                                   static_cast<T*>(u[i]), dims_of(pl));
            }
            HIP_TRY(hipGetLastError(), "batch unpack launch");
            return ETD_OK;
        }();
        if (fork) {
            // join every forked group back to the caller's stream, also after an error
            const hipError_t e1 = hipEventRecord(G.done, gs);
            const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s, G.done, 0) : e1;
            if (st == ETD_OK && e2 != hipSuccess) st = hip_fail(e2, "batch join");
        }
        if (st != ETD_OK) return st;
    }
    return ETD_OK;
}

template <typename M, int NC>
etd_status batch_autotune_t(Batch& B, char* ws, hipStream_t s) {
    typedef typename M::elem T;
    for (BatchGroup& G : B.groups) {
        const long nlines = long(G.np[1]) * G.np[2];
        for (int stage = 0; stage < B.dim; ++stage) {
            const int d = stage == B.dim - 1 ? 0 : (B.dim == 3 ? (stage == 0 ? 2 : 1) : 1);
            const int st_kind = stage == B.dim - 1 ? 2 : stage;
            const std::vector<TileShape> cand =
                d == 0 ? x_candidates<T, NC>(G.np[0], nlines) : outer_candidates<T, NC>(G.np[d]);
            TileShape best{};
            float best_ms = 0.f;
            for (TileShape t : cand) {
                G.tile[d] = t;
                TRY(upload_descriptors(B, ws, s));
                float ms = 0.f;
                TRY(time_launches([&]() { return group_stage<M, NC>(B, G, st_kind, ws, 0.0, 0, s); }, kTuneReps, s, ms));
                if (best.rb == 0 || ms < best_ms) {
                    best = t;
                    best_ms = ms;
                }
            }
            G.tile[d] = best;
        }
    }
    return upload_descriptors(B, ws, s);
}

}  // namespace
