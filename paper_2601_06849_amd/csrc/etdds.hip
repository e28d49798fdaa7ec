// Spectral ETD2RK-DS stepper for gfx950: stage kernels and the C ABI.
//
// One step of the Pade-based scheme (Sec. 3.1; Algorithms 1-2), written in the
// increment form Q(z) g = Q(0) g + P diag(Q(tau lambda) - Q(0)) P g, with P
// the symmetric orthogonal eigenvector matrix of the direction (so the forward
// product P^T and the backward product P are the same matrix):
//
//   outer stage(s)  (3-D: z then y; 2-D: y)
//       w_a = g_a + P diag(q1 - 1) P g_a      for g = [U, f(t_n, U)] (first)
//                                              or g = [w1, w2]       (middle)
//   x stage (fused, Algorithm 2 steps 3.5.1-3.5.7)
//       c   = (q1 - 1) .* (P w3) + tau (q2 - 1) .* (P w4)
//       W   = w3 + tau w4 + P c
//       d   = f(t_{n+1}, W) - w4
//       U+  = W + tau d / 2 + tau P ((q3 - 1/2) .* (P d))
//
// which is Q1 w3 + tau Q2 w4 and W + tau Q3 (F1 - w4) rearranged.  Every
// product is a dense mode-d contraction with P and runs on the MFMA units
// (FP64 or FP32 16x16x4).  A workgroup owns a tile of 16 grid lines (x stage)
// or 16 columns (outer stages) over the whole contracted direction, so the
// forward product, the Hadamard scaling and the backward product stay on chip.
//
// This file holds the C ABI.  The kernels and host drivers are in the headers
// of library.hpp; each mode-product precision instantiates them in a
// translation unit of its own (kern_<precision>.hip), reached here through
// its table of entry functions (PrecisionOps).
#include "library.hpp"

namespace etdds {
thread_local std::string g_err;
}  // namespace etdds

struct etd_plan {
    Plan p;
    mutable StageTimer timer;
    unsigned long long serial = 0;   // unique per plan (workspace registry)
};

struct etd_batch {
    Batch b;
};

struct etd_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::shared_ptr<unsigned> generation;   // batch graphs: the batch's token
    unsigned captured = 0;                  // its value at capture
};

namespace {

// The plan whose tables each workspace holds: etd_plan_upload records the
// workspace address with the plan's serial number, and every call that takes
// a plan workspace checks it, so a workspace that was never uploaded, or was
// last uploaded for another plan, is refused instead of yielding garbage
// tables (or, undersized, stage writes beyond its end).
std::mutex g_ws_mutex;
std::unordered_map<const void*, unsigned long long> g_ws_owner;
std::atomic<unsigned long long> g_plan_serial{0};

etd_status check_uploaded(const etd_plan* plan, const void* ws) {
    std::lock_guard<std::mutex> lk(g_ws_mutex);
    const auto it = g_ws_owner.find(ws);
    if (it == g_ws_owner.end() || it->second != plan->serial)
        return fail(ETD_EWORKSPACE, "workspace was not uploaded for this plan (etd_plan_upload)");
    return ETD_OK;
}

// check_ws (pointer and alignment), then the upload record
etd_status check_plan_ws(const etd_plan* plan, const void* ws) {
    const etd_status st = check_ws(plan->p, ws);
    return st != ETD_OK ? st : check_uploaded(plan, ws);
}

const PrecisionOps& ops_for(int precision) {
    switch (precision) {
    case ETD_FP64: return ops_fp64();
    case ETD_FP32: return ops_fp32();
    case ETD_FP64_FP32: return ops_fp64_fp32();
    case ETD_FP64_BF16X6: return ops_fp64_bf16x6();
    default: return ops_bf16x6();
    }
}

etd_status batch_dispatch_advance(Batch& B, void* const* u, double t0, int nsteps, char* ws, hipStream_t s) {
    return ops_for(B.precision).batch_advance(B, u, t0, nsteps, ws, s);
}

etd_status resolve_tile_any(const Plan& pl, int d, TileShape t, TileShape& out, long copies = 1) {
    return ops_for(pl.prob.precision).resolve_tile(pl, d, t, out, copies);
}

etd_status batch_check(const Batch& B, void* const* u, int nsteps, const void* ws) {
    if (!u) return fail(ETD_EINVAL, "field pointer array is NULL");
    for (size_t i = 0; i < B.plans.size(); ++i)
        if (!u[i]) return fail(ETD_EINVAL, "a field pointer is NULL");
    if (nsteps < 0) return fail(ETD_EINVAL, "nsteps must be >= 0");
    if (!ws || ws != B.uploaded) return fail(ETD_EWORKSPACE, "workspace is not the one the batch was uploaded to");
    return ETD_OK;
}

// The validation reductions of etd_compare: per-block partials into part
// (kRedBlocks x 4 doubles), then the four results into res (device).
etd_status compare_enqueue(const Plan& pl, const void* a, const void* b, double* part, double* res, hipStream_t s) {
    const long n = long(pl.nc) * pl.n[0] * pl.n[1] * pl.n[2];
    if (pl.elem == 8)
        hipLaunchKernelGGL(compare_partial<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, s,
                           static_cast<const double*>(a), static_cast<const double*>(b), n, part);
    else
        hipLaunchKernelGGL(compare_partial<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, s,
                           static_cast<const float*>(a), static_cast<const float*>(b), n, part);
    HIP_TRY(hipGetLastError(), "compare launch");
    hipLaunchKernelGGL(compare_final, dim3(1), dim3(kRedThreads), 0, s, part, kRedBlocks, res);
    HIP_TRY(hipGetLastError(), "compare final launch");
    return ETD_OK;
}

// Partial sums of etd_compare_noalloc: a fixed device array (one copy per
// GPU, held until the process ends).  The grid-stride reduction writes
// exactly kRedBlocks x 4 partials whatever the field size, and every call
// overwrites all of them before reading, so nothing needs clearing; calls
// that overlap on one GPU share the array and race.
constexpr int kScratchDoubles = kRedBlocks * 4;
static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` per device ordinal, looked up once per device
// with that device current (the array's host-side name is not a device
// address).
std::mutex g_scratch_mutex;
std::vector<double*> g_scratch_ptr;

etd_status scratch_on_current_device(double** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "current device");
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (dev >= int(g_scratch_ptr.size())) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (!p) return fail(ETD_EHIP, "scratch symbol address: NULL");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return ETD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

etd_status etd_plan_create(const etd_problem* prob, etd_plan** out) {
    if (!prob || !out) return fail(ETD_EINVAL, "NULL argument");
    *out = nullptr;
    etd_plan* p = new (std::nothrow) etd_plan;
    if (!p) return fail(ETD_EINVAL, "out of host memory");
    std::string err;
    const etd_status st = build_plan(*prob, p->p, err);
    if (st != ETD_OK) {
        delete p;
        return fail(st, err);
    }
    p->serial = ++g_plan_serial;
    *out = p;
    return ETD_OK;
}

etd_status etd_plan_workspace_bytes(const etd_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return fail(ETD_EINVAL, "NULL argument");
    *bytes = plan->p.lay.total;
    return ETD_OK;
}

etd_status etd_plan_upload(const etd_plan* plan, void* ws, size_t bytes, void* stream) {
    if (!plan) return fail(ETD_EINVAL, "NULL plan");
    etd_status st = check_ws(plan->p, ws);
    if (st != ETD_OK) return st;
    if (bytes < plan->p.lay.total) return fail(ETD_EWORKSPACE, "workspace smaller than etd_plan_workspace_bytes()");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(ws, plan->p.image.data(), plan->p.table_bytes, hipMemcpyHostToDevice, s), "table upload");
    // The stage buffers start zeroed so that padded lanes are exact zeros
    // before the first pack.
    HIP_TRY(hipMemsetAsync(static_cast<char*>(ws) + plan->p.lay.field[0], 0,
                           plan->p.lay.total - plan->p.lay.field[0], s),
            "workspace clear");
    // The host image must outlive the asynchronous copy.
    HIP_TRY(hipStreamSynchronize(s), "table upload sync");
    std::lock_guard<std::mutex> lk(g_ws_mutex);
    g_ws_owner[ws] = plan->serial;
    return ETD_OK;
}

etd_status etd_advance(const etd_plan* plan, void* u, double t0, int nsteps, void* ws, void* stream) {
    if (!plan) return fail(ETD_EINVAL, "NULL plan");
    if (nsteps < 0) return fail(ETD_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(t0)) return fail(ETD_EINVAL, "t0 must be finite");
    if (!u) return fail(ETD_EINVAL, "field pointer is NULL");
    etd_status st = check_ws(plan->p, ws);
    if (st != ETD_OK) return st;
    if (nsteps == 0) return ETD_OK;
    st = check_uploaded(plan, ws);
    if (st != ETD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    return ops_for(plan->p.prob.precision).advance(plan->p, plan->timer, u, t0, nsteps, w, s);
}

etd_status etd_adjoint_workspace_bytes(const etd_plan* plan, int nsteps, size_t* bytes) {
    if (!plan || !bytes) return fail(ETD_EINVAL, "NULL argument");
    if (nsteps < 1) return fail(ETD_EINVAL, "nsteps must be >= 1");
    const etd_status st = adjoint_supported(plan->p);
    if (st != ETD_OK) return st;
    *bytes = adjoint_layout(plan->p, nsteps).total;
    return ETD_OK;
}

etd_status etd_adjoint_workspace_bytes_segment(const etd_plan* plan, int nsteps, int segment, size_t* bytes) {
    if (!plan || !bytes) return fail(ETD_EINVAL, "NULL argument");
    if (nsteps < 1) return fail(ETD_EINVAL, "nsteps must be >= 1");
    if (segment < min_segment(nsteps) || segment > nsteps)
        return fail(ETD_EINVAL, "segment must lie between ceil(sqrt(nsteps)) and nsteps");
    const etd_status st = adjoint_supported(plan->p);
    if (st != ETD_OK) return st;
    *bytes = adjoint_layout(plan->p, nsteps, segment).total;
    return ETD_OK;
}

etd_status etd_adjoint(const etd_plan* plan, const void* u0, double t0, int nsteps, const void* ubar_final,
                       void* ubar0, double* grad, void* ws, void* adj_ws, size_t adj_bytes, void* stream) {
    if (!plan || !u0 || !ubar_final || !ubar0 || !grad) return fail(ETD_EINVAL, "NULL argument");
    if (nsteps < 1) return fail(ETD_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(t0)) return fail(ETD_EINVAL, "t0 must be finite");
    etd_status st = check_plan_ws(plan, ws);
    if (st != ETD_OK) return st;
    st = adjoint_supported(plan->p);
    if (st != ETD_OK) return st;
    const int segment = adjoint_segment_for(plan->p, nsteps, adj_bytes);
    const AdjLayout L = adjoint_layout(plan->p, nsteps, segment);
    if (!adj_ws || reinterpret_cast<uintptr_t>(adj_ws) % 256 != 0)
        return fail(ETD_EWORKSPACE, "adjoint workspace must be non-NULL and 256-byte aligned");
    if (adj_bytes < L.total) return fail(ETD_EWORKSPACE, "adjoint workspace smaller than etd_adjoint_workspace_bytes()");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    char* a = static_cast<char*>(adj_ws);
    const Plan& pl = plan->p;
    return ops_for(pl.prob.precision).adjoint(pl, plan->timer, u0, t0, nsteps, segment, ubar_final, ubar0, grad, w, a,
                                              s);
}

etd_status etd_plan_autotune(etd_plan* plan, void* ws, void* stream) {
    if (!plan) return fail(ETD_EINVAL, "NULL plan");
    etd_status st = check_plan_ws(plan, ws);
    if (st != ETD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    Plan& pl = plan->p;
    const bool timing = plan->timer.on;
    plan->timer.on = false;
    st = ops_for(pl.prob.precision).autotune(pl, w, s);
    plan->timer.on = timing;
    return st;
}

etd_status etd_plan_tiles(const etd_plan* plan, int tiles[6]) {
    if (!plan || !tiles) return fail(ETD_EINVAL, "NULL argument");
    const Plan& pl = plan->p;
    for (int d = 0; d < 3; ++d) {
        TileShape t{};
        if (d < pl.dim) {
            const etd_status st = resolve_tile_any(pl, d, TileShape{pl.tile_rb[d], pl.tile_cb[d]}, t);
            if (st != ETD_OK) return st;
        }
        tiles[2 * d] = t.rb;
        tiles[2 * d + 1] = t.cb;
    }
    return ETD_OK;
}

etd_status etd_plan_set_tiles(etd_plan* plan, const int tiles[6]) {
    if (!plan || !tiles) return fail(ETD_EINVAL, "NULL argument");
    Plan& pl = plan->p;
    TileShape r[3];
    for (int d = 0; d < pl.dim; ++d) {
        const etd_status st = resolve_tile_any(pl, d, TileShape{tiles[2 * d], tiles[2 * d + 1]}, r[d]);
        if (st != ETD_OK) return st;
    }
    for (int d = 0; d < pl.dim; ++d) {
        const bool dflt = tiles[2 * d] == 0 && tiles[2 * d + 1] == 0;
        pl.tile_rb[d] = dflt ? 0 : r[d].rb;
        pl.tile_cb[d] = dflt ? 0 : r[d].cb;
    }
    return ETD_OK;
}

etd_status etd_plan_set_schedule(etd_plan* plan, int schedule) {
    if (!plan) return fail(ETD_EINVAL, "NULL plan");
    if (schedule != ETD_SCHEDULE_AUTO && schedule != ETD_SCHEDULE_STAGES && schedule != ETD_SCHEDULE_RESIDENT)
        return fail(ETD_EINVAL, "schedule must be ETD_SCHEDULE_AUTO, _STAGES or _RESIDENT");
    if (schedule == ETD_SCHEDULE_RESIDENT && !resident_eligible(plan->p))
        return fail(ETD_EUNSUPPORTED, "the resident schedule needs one padded extent of at most 128 in every direction");
    plan->p.schedule = schedule;
    return ETD_OK;
}

etd_status etd_plan_schedule(const etd_plan* plan, int* schedule) {
    if (!plan || !schedule) return fail(ETD_EINVAL, "NULL argument");
    const Plan& pl = plan->p;
    *schedule = pl.schedule == ETD_SCHEDULE_RESIDENT && resident_eligible(pl) ? ETD_SCHEDULE_RESIDENT
                                                                               : ETD_SCHEDULE_STAGES;
    return ETD_OK;
}

// A batch offers no table query and uploads only the packed image, so the
// FP64 host tables of its instances (an n_d x n_d matrix per direction) are
// dropped once the image is built.
static void release_host_tables(Plan& pl) {
    for (int d = 0; d < 3; ++d) {
        std::vector<double>().swap(pl.P[d]);
        for (int c = 0; c < 2; ++c) {
            std::vector<double>().swap(pl.lam[d][c]);
            for (int l = 0; l < 3; ++l) {
                std::vector<double>().swap(pl.rat[d][c][l]);
                std::vector<double>().swap(pl.inc[d][c][l]);
            }
        }
    }
}

etd_status etd_batch_create(const etd_problem* probs, int count, etd_batch** out) {
    if (!probs || !out) return fail(ETD_EINVAL, "NULL argument");
    *out = nullptr;
    if (count < 1 || count > kMaxBatch) return fail(ETD_EINVAL, "count must be in 1..4096");
    etd_batch* b = new (std::nothrow) etd_batch;
    if (!b) return fail(ETD_EINVAL, "out of host memory");
    Batch& B = b->b;
    B.plans.resize(count);
    for (int i = 0; i < count; ++i) {
        std::string err;
        const etd_status st = build_plan(probs[i], B.plans[i], err);
        if (st != ETD_OK) {
            delete b;
            return fail(st, "instance " + std::to_string(i) + ": " + err);
        }
        const Plan& pl = B.plans[i];
        if (i == 0) {
            B.dim = pl.dim;
            B.nc = pl.nc;
            B.precision = pl.prob.precision;
        } else if (pl.dim != B.dim || pl.nc != B.nc || pl.prob.precision != B.precision) {
            delete b;
            return fail(ETD_EINVAL, "instance " + std::to_string(i) +
                                        ": a batch takes one dimension, component count and precision");
        }
        release_host_tables(B.plans[i]);
        bool fused = x_fused(pl.np[0], pl.nc, pl.elem);
        for (int d = 1; d < pl.dim; ++d) fused = fused && outer_fused(pl.np[d], pl.nc, pl.elem);
        if (!fused) {
            delete b;
            return fail(ETD_EUNSUPPORTED, "instance " + std::to_string(i) +
                                              ": its two-component tile exceeds the LDS (single plans only)");
        }
    }
    batch_layout(B);
    for (BatchGroup& G : B.groups) {
        const Plan& pl = B.plans[G.inst[0]];
        for (int d = 0; d < pl.dim; ++d) {
            const etd_status st = resolve_tile_any(pl, d, TileShape{}, G.tile[d], long(G.inst.size()));
            if (st != ETD_OK) {
                delete b;
                return st;
            }
        }
    }
    *out = b;
    return ETD_OK;
}

etd_status etd_batch_workspace_bytes(const etd_batch* batch, size_t* bytes) {
    if (!batch || !bytes) return fail(ETD_EINVAL, "NULL argument");
    *bytes = batch->b.total;
    return ETD_OK;
}

etd_status etd_batch_upload(etd_batch* batch, void* ws, size_t bytes, void* stream) {
    if (!batch) return fail(ETD_EINVAL, "NULL batch");
    Batch& B = batch->b;
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(ETD_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    if (bytes < B.total) return fail(ETD_EWORKSPACE, "workspace smaller than etd_batch_workspace_bytes()");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    for (size_t i = 0; i < B.plans.size(); ++i) {
        const Plan& pl = B.plans[i];
        const size_t skip = B.skip[i];   // P tables borrowed from an earlier instance
        HIP_TRY(hipMemcpyAsync(w + B.base[i] + skip, pl.image.data() + skip, pl.table_bytes - skip,
                               hipMemcpyHostToDevice, s),
                "table upload");
        HIP_TRY(hipMemsetAsync(w + B.base[i] + pl.lay.field[0], 0, pl.lay.total - pl.lay.field[0], s),
                "workspace clear");
    }
    HIP_TRY(hipStreamSynchronize(s), "table upload sync");
    if (!B.fork) HIP_TRY(hipEventCreateWithFlags(&B.fork, hipEventDisableTiming), "batch event");
    for (BatchGroup& G : B.groups) {
        if (!G.stream) HIP_TRY(hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking), "batch stream");
        if (!G.done) HIP_TRY(hipEventCreateWithFlags(&G.done, hipEventDisableTiming), "batch event");
    }
    return upload_descriptors(B, w, s);
}

etd_status etd_batch_advance(etd_batch* batch, void* const* u, double t0, int nsteps, void* ws, void* stream) {
    if (!batch) return fail(ETD_EINVAL, "NULL batch");
    if (!std::isfinite(t0)) return fail(ETD_EINVAL, "t0 must be finite");
    Batch& B = batch->b;
    etd_status st = batch_check(B, u, nsteps, ws);
    if (st != ETD_OK) return st;
    if (nsteps == 0) return ETD_OK;
    return batch_dispatch_advance(B, u, t0, nsteps, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

etd_status etd_batch_autotune(etd_batch* batch, void* ws, void* stream) {
    if (!batch) return fail(ETD_EINVAL, "NULL batch");
    Batch& B = batch->b;
    if (!ws || ws != B.uploaded) return fail(ETD_EWORKSPACE, "workspace is not the one the batch was uploaded to");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    return ops_for(B.precision).batch_autotune(B, w, s);
}

etd_status etd_batch_tiles(const etd_batch* batch, int instance, int tiles[6]) {
    if (!batch || !tiles) return fail(ETD_EINVAL, "NULL argument");
    const Batch& B = batch->b;
    if (instance < 0 || instance >= int(B.plans.size())) return fail(ETD_EINVAL, "instance out of range");
    for (const BatchGroup& G : B.groups)
        for (int i : G.inst)
            if (i == instance) {
                for (int d = 0; d < 3; ++d) {
                    tiles[2 * d] = d < B.dim ? G.tile[d].rb : 0;
                    tiles[2 * d + 1] = d < B.dim ? G.tile[d].cb : 0;
                }
                return ETD_OK;
            }
    return fail(ETD_EINVAL, "instance not found");
}

etd_status etd_batch_groups(const etd_batch* batch, int* groups) {
    if (!batch || !groups) return fail(ETD_EINVAL, "NULL argument");
    *groups = int(batch->b.groups.size());
    return ETD_OK;
}

etd_status etd_batch_destroy(etd_batch* batch) {
    if (!batch) return ETD_OK;
    Batch& B = batch->b;
    for (BatchGroup& G : B.groups) {
        if (G.stream) (void)hipStreamDestroy(G.stream);
        if (G.done) (void)hipEventDestroy(G.done);
    }
    if (B.fork) (void)hipEventDestroy(B.fork);
    *B.generation = 0;
    delete batch;
    return ETD_OK;
}

etd_status etd_graph_capture(const etd_plan* plan, void* u, double t0, int nsteps, void* ws, void* stream,
                             etd_graph** out) {
    if (!plan || !out || !u) return fail(ETD_EINVAL, "NULL argument");
    *out = nullptr;
    if (!stream) return fail(ETD_EINVAL, "graph capture needs a stream other than the default stream");
    if (nsteps < 1) return fail(ETD_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(t0)) return fail(ETD_EINVAL, "t0 must be finite");
    etd_status st = check_plan_ws(plan, ws);
    if (st != ETD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool timing = plan->timer.on;
    plan->timer.on = false;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "graph capture begin");
    char* w = static_cast<char*>(ws);
    st = ops_for(plan->p.prob.precision).advance(plan->p, plan->timer, u, t0, nsteps, w, s);
    plan->timer.on = timing;
    hipGraph_t g;
    st = end_capture(s, st, g);
    if (st != ETD_OK) return st;
    etd_graph* G = new (std::nothrow) etd_graph;
    if (!G) {
        (void)hipGraphDestroy(g);
        return fail(ETD_EINVAL, "out of host memory");
    }
    G->graph = g;
    const hipError_t he = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (he != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete G;
        return hip_fail(he, "graph instantiate");
    }
    *out = G;
    return ETD_OK;
}

etd_status etd_batch_graph_capture(etd_batch* batch, void* const* u, double t0, int nsteps, void* ws, void* stream,
                                   etd_graph** out) {
    if (!batch || !out) return fail(ETD_EINVAL, "NULL argument");
    *out = nullptr;
    if (!stream) return fail(ETD_EINVAL, "graph capture needs a stream other than the default stream");
    if (nsteps < 1) return fail(ETD_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(t0)) return fail(ETD_EINVAL, "t0 must be finite");
    Batch& B = batch->b;
    etd_status st = batch_check(B, u, nsteps, ws);
    if (st != ETD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "graph capture begin");
    st = batch_dispatch_advance(B, u, t0, nsteps, static_cast<char*>(ws), s);
    hipGraph_t g;
    st = end_capture(s, st, g);
    if (st != ETD_OK) return st;
    etd_graph* G = new (std::nothrow) etd_graph;
    if (!G) {
        (void)hipGraphDestroy(g);
        return fail(ETD_EINVAL, "out of host memory");
    }
    G->graph = g;
    G->generation = B.generation;
    G->captured = *B.generation;
    const hipError_t he = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (he != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete G;
        return hip_fail(he, "graph instantiate");
    }
    *out = G;
    return ETD_OK;
}

etd_status etd_graph_launch(etd_graph* graph, void* stream) {
    if (!graph || !graph->exec) return fail(ETD_EINVAL, "NULL graph");
    if (graph->generation && *graph->generation != graph->captured)
        return fail(ETD_EINVAL, "graph is stale: its batch was re-tuned, re-uploaded or destroyed since capture");
    HIP_TRY(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)), "graph launch");
    return ETD_OK;
}

etd_status etd_graph_destroy(etd_graph* graph) {
    if (!graph) return ETD_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return ETD_OK;
}

etd_status etd_compare(const etd_plan* plan, const void* a, const void* b, double out[4], void* ws, void* stream) {
    if (!plan || !a || !b || !out) return fail(ETD_EINVAL, "NULL argument");
    etd_status st = check_plan_ws(plan, ws);
    if (st != ETD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + plan->p.lay.reduce);
    st = compare_enqueue(plan->p, a, b, part, part + kRedBlocks * 4, s);
    if (st != ETD_OK) return st;
    HIP_TRY(hipMemcpyAsync(out, part + kRedBlocks * 4, 4 * sizeof(double), hipMemcpyDeviceToHost, s), "compare copy");
    HIP_TRY(hipStreamSynchronize(s), "compare sync");
    if (out[3] > 0) return fail(ETD_ENONFINITE, "field holds non-finite values");
    return ETD_OK;
}

etd_status etd_compare_noalloc(const etd_plan* plan, const void* a, const void* b, double* out_dev, void* stream) {
    if (!plan || !a || !b || !out_dev) return fail(ETD_EINVAL, "NULL argument");
    double* part = nullptr;
    etd_status st = scratch_on_current_device(&part);
    if (st != ETD_OK) return st;
    return compare_enqueue(plan->p, a, b, part, out_dev, static_cast<hipStream_t>(stream));
}

etd_status etd_plan_problem(const etd_plan* plan, etd_problem* out) {
    if (!plan || !out) return fail(ETD_EINVAL, "NULL argument");
    *out = plan->p.prob;
    return ETD_OK;
}

etd_status etd_plan_table(const etd_plan* plan, int which, int d, int comp, double* out, size_t count) {
    if (!plan || !out) return fail(ETD_EINVAL, "NULL argument");
    const Plan& pl = plan->p;
    if (d < 0 || d >= pl.dim || comp < 0 || comp >= pl.nc) return fail(ETD_EINVAL, "direction or component out of range");
    const std::vector<double>* src = nullptr;
    if (which == 0) src = &pl.lam[d][comp];
    else if (which == 1) src = &pl.P[d];
    else if (which >= 2 && which <= 4) src = &pl.rat[d][comp][which - 2];
    else if (which >= 5 && which <= 7) src = &pl.inc[d][comp][which - 5];
    else return fail(ETD_EINVAL, "unknown table");
    if (count < src->size()) return fail(ETD_EINVAL, "output buffer too small");
    std::memcpy(out, src->data(), src->size() * sizeof(double));
    return ETD_OK;
}

etd_status etd_timing_enable(etd_plan* plan, int enable) {
    if (!plan) return fail(ETD_EINVAL, "NULL plan");
    plan->timer.on = enable != 0;
    plan->timer.used = 0;
    plan->timer.kind.clear();
    return ETD_OK;
}

etd_status etd_timing_read(etd_plan* plan, double ms[3], long long counts[3]) {
    if (!plan || !ms || !counts) return fail(ETD_EINVAL, "NULL argument");
    StageTimer& t = plan->timer;
    for (int k = 0; k < 3; ++k) {
        ms[k] = 0.0;
        counts[k] = 0;
    }
    if (t.used > 0) HIP_TRY(hipEventSynchronize(t.pool[t.used - 1]), "timing sync");
    for (size_t i = 0; i < t.kind.size(); ++i) {
        float dt = 0.0f;
        HIP_TRY(hipEventElapsedTime(&dt, t.pool[2 * i], t.pool[2 * i + 1]), "timing elapsed");
        ms[t.kind[i]] += dt;
        counts[t.kind[i]] += 1;
    }
    t.used = 0;
    t.kind.clear();
    return ETD_OK;
}

etd_status etd_plan_destroy(etd_plan* plan) {
    if (plan) {
        for (hipEvent_t e : plan->timer.pool) (void)hipEventDestroy(e);
        std::lock_guard<std::mutex> lk(g_ws_mutex);
        for (auto it = g_ws_owner.begin(); it != g_ws_owner.end();)
            it = it->second == plan->serial ? g_ws_owner.erase(it) : std::next(it);
    }
    delete plan;
    return ETD_OK;
}

const char* etd_status_string(etd_status s) {
    switch (s) {
    case ETD_OK: return "ok";
    case ETD_EINVAL: return "invalid argument";
    case ETD_EUNSUPPORTED: return "unsupported configuration";
    case ETD_EWORKSPACE: return "bad workspace";
    case ETD_EHIP: return "HIP runtime error";
    case ETD_ENONFINITE: return "non-finite values";
    }
    return "unknown status";
}

const char* etd_last_error(void) { return g_err.c_str(); }

}  // extern "C"
