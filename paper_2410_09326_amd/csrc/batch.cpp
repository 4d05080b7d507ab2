// Batched executor: many small, uneven circuits (parameter sweeps, paper
// Sec. IV-E) in one graph launch.  Circuits whose whole state fits in one
// work-group's LDS run start to finish in one kernel (one work-group each);
// the larger ones are planned into tile passes (register tiles, or LDS tiles
// where a pass holds dense blocks) and pass p of every circuit that has one
// runs in the graph nodes of step p, one node per kernel kind.  <Z_i> of
// every circuit is reduced on the device in FP64 and read back once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"

using namespace qops;

struct qops_batch_exec {
    int prec = 0;
    int count = 0;
    int small_max_n = 0, tile_bits = 0, fuse_k = 1;
    std::vector<int> n;
    std::vector<qops::Plan> plans;
    std::vector<BatchCirc> circs;
    std::vector<int32_t> small_ids, big_ids;
    struct Node {                       // one kernel of step `pass`
        int pass = 0;
        int kind = 0;                   // 0: register tiles (R, W), 1: LDS tiles
        int R = 0, W = 0;
        int lds = 0;                    // dynamic LDS bytes
        std::vector<BatchItem> items;
        BatchItem* d = nullptr;
    };
    std::vector<Node> nodes;
    std::vector<BatchItem> z_items;
    std::vector<size_t> coef_base;      // offset of each plan's coefficients in the batch image
    std::vector<size_t> state_base;     // byte offset of each tile-pass circuit's state
    size_t total_out = 0, total_part = 0, total_state_bytes = 0;
    int lds_small = 0, grid = 0;
    // device
    BatchCirc* d_circs = nullptr;
    PassHdr* d_hdrs = nullptr;
    DevOp* d_ops = nullptr;
    void* d_coef = nullptr;
    int32_t* d_small = nullptr;
    int32_t* d_big = nullptr;
    BatchItem* d_zitems = nullptr;
    double* d_part = nullptr;
    double* d_out = nullptr;
    char* d_states = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double last_seconds = 0;
};

namespace {

int32_t plan_all(qops_batch_exec* e, const qops_batch* b)
{
    e->plans.resize(b->count);
    for (int i = 0; i < b->count; ++i) {
        const int n = b->n[i];
        if (n < 1 || n > 26) return set_error(QOPS_UNSUPPORTED, "batch circuits need 1 <= n <= 26");
        PlanParams par = params_from(nullptr, n, b->precision);
        par.state_lds_max_n = e->small_max_n;
        par.max_fuse_k = e->fuse_k;
        par.L_lds = std::min(e->tile_bits, n);
        // register tiles of the same width: up to 5 (complex64) / 4
        // (complex128) register bits, the rest wave bits
        par.R = b->precision == QOPS_C64 ? 5 : 4;
        par.W = std::max(0, std::min(2, std::min(e->tile_bits, n) - 6 - par.R));
        Err er = build_plan(n, b->precision, nullptr, b->gates[i], b->n_gates[i], par, e->plans[i]);
        if (!er.ok()) return set_error(er.code, "circuit " + std::to_string(i) + ": " + er.msg);
        const Plan& p = e->plans[i];
        for (const PassPlan& pp : p.passes) {
            const bool ok = n <= e->small_max_n ? pp.type == PASS_STATE_LDS
                                                : (pp.type == PASS_TILE_LDS || pp.type == PASS_TILE_REG);
            if (!ok)
                return set_error(QOPS_UNSUPPORTED, "circuit " + std::to_string(i) +
                                                       ": needs an operation the batched executor does not run "
                                                       "(physical swap or a dense block too wide for its tile)");
        }
    }
    return QOPS_OK;
}

template <typename T>
void cast_coef(const std::vector<double>& src, std::vector<unsigned char>& dst, size_t at)
{
    T* d = reinterpret_cast<T*>(dst.data()) + at;
    for (size_t i = 0; i < src.size(); ++i) d[i] = (T)src[i];
}

int32_t layout(qops_batch_exec* e)
{
    const size_t asz = e->prec == QOPS_C64 ? 8 : 16, csz = asz / 2;
    std::vector<PassHdr> hdrs;
    std::vector<DevOp> ops;
    size_t coef_n = 0;
    e->coef_base.assign(e->count, 0);
    e->state_base.assign(e->count, 0);
    e->circs.assign(e->count, BatchCirc{});
    e->small_ids.clear();
    e->big_ids.clear();
    size_t out0 = 0, part0 = 0, state_off = 0;
    int maxpass = 0, max_small_n = 1;
    for (int i = 0; i < e->count; ++i) {
        const Plan& p = e->plans[i];
        BatchCirc& c = e->circs[i];
        c.n = p.n;
        c.out0 = (int32_t)out0;
        out0 += p.n;
        e->coef_base[i] = coef_n;
        const int op_base = (int)ops.size();
        for (DevOp d : p.dops) {
            // LDS-tile ops with b = 1 address the pass's staged coefficients
            const bool staged = d.b && (d.type == OP_MFMA || d.type == OP_DIAG_LDS || d.type == OP_DENSE_LDS);
            d.coef += staged ? 0 : (int32_t)coef_n;
            ops.push_back(d);
        }
        if (p.n <= e->small_max_n) {
            c.op0 = op_base + (p.passes.empty() ? 0 : p.passes[0].op0);
            c.nops = p.passes.empty() ? 0 : p.passes[0].nops;
            c.npass = 0;
            e->small_ids.push_back(i);
            max_small_n = std::max(max_small_n, p.n);
        } else {
            c.hdr0 = (int32_t)hdrs.size();
            c.npass = (int32_t)p.passes.size();
            for (const PassPlan& pp : p.passes) {
                PassHdr h = p.hdrs[pp.hdr];
                h.op0 += op_base;
                h.coef_src += (int32_t)coef_n;
                hdrs.push_back(h);
            }
            maxpass = std::max(maxpass, c.npass);
            c.part0 = (int32_t)part0;
            const int s = std::min(p.n, 13);
            part0 += (size_t)1 << (p.n - s);
            e->state_base[i] = state_off;      // pointer filled in after the allocation
            state_off += ((size_t)1 << p.n) * asz;
            e->big_ids.push_back(i);
        }
        coef_n += p.coef.size();
    }
    e->total_out = out0;
    e->total_part = part0;
    e->total_state_bytes = state_off;
    e->lds_small = (int)(((size_t)1 << max_small_n) * asz);
    e->grid = device_cus() * 2;
    // work lists: pass p of every circuit that has it, one list per kernel
    // kind (register tiles of each R/W split, LDS tiles); the reduction chunks
    e->nodes.clear();
    e->z_items.clear();
    for (int ps = 0; ps < maxpass; ++ps) {
        const size_t first = e->nodes.size();
        for (int i : e->big_ids) {
            const BatchCirc& c = e->circs[i];
            const Plan& p = e->plans[i];
            if (ps >= c.npass) continue;
            const PassPlan& pp = p.passes[ps];
            const PassHdr& h = p.hdrs[pp.hdr];
            const int kind = pp.type == PASS_TILE_REG ? 0 : 1;
            const int R = kind == 0 ? pp.R : 0, W = kind == 0 ? pp.W : 0;
            size_t at = first;
            while (at < e->nodes.size() &&
                   !(e->nodes[at].kind == kind && e->nodes[at].R == R && e->nodes[at].W == W))
                ++at;
            if (at == e->nodes.size()) {
                qops_batch_exec::Node nd;
                nd.pass = ps;
                nd.kind = kind;
                nd.R = R;
                nd.W = W;
                e->nodes.push_back(nd);
            }
            qops_batch_exec::Node& nd = e->nodes[at];
            const int need = kind == 0 ? h.lds_bytes
                                       : (int)(((size_t)1 << h.L) * asz + (size_t)h.coef_n * csz);
            nd.lds = std::max(nd.lds, (need + 15) & ~15);
            const int nt = 1 << (p.n - pp.L);
            for (int t = 0; t < nt; ++t) nd.items.push_back(BatchItem{i, t});
        }
    }
    for (const auto& nd : e->nodes)
        if (nd.lds > 160 * 1024) return set_error(QOPS_UNSUPPORTED, "batch pass needs more LDS than a CU has");
    for (int i : e->big_ids) {
        const Plan& p = e->plans[i];
        const int s = std::min(p.n, 13);
        for (int t = 0; t < (1 << (p.n - s)); ++t) e->z_items.push_back(BatchItem{i, t});
    }
    // coefficient image in the state precision
    std::vector<unsigned char> cimg(std::max<size_t>(coef_n, 1) * csz);
    for (int i = 0; i < e->count; ++i) {
        if (e->prec == QOPS_C64) cast_coef<float>(e->plans[i].coef, cimg, e->coef_base[i]);
        else cast_coef<double>(e->plans[i].coef, cimg, e->coef_base[i]);
    }
    // device buffers
    auto up = [&](auto*& dptr, const void* src, size_t bytes) -> hipError_t {
        hipError_t er = hipMalloc((void**)&dptr, std::max<size_t>(bytes, 64));
        if (er == hipSuccess && bytes) er = hipMemcpy(dptr, src, bytes, hipMemcpyHostToDevice);
        return er;
    };
    hipError_t er = hipMalloc((void**)&e->d_states, std::max<size_t>(state_off, 64));
    if (er != hipSuccess) return hip_fail(er, "batch state allocation");
    for (int i : e->big_ids) e->circs[i].state = e->d_states + e->state_base[i];
    if ((er = up(e->d_circs, e->circs.data(), e->circs.size() * sizeof(BatchCirc))) != hipSuccess ||
        (er = up(e->d_hdrs, hdrs.data(), hdrs.size() * sizeof(PassHdr))) != hipSuccess ||
        (er = up(e->d_ops, ops.data(), ops.size() * sizeof(DevOp))) != hipSuccess ||
        (er = up(e->d_coef, cimg.data(), cimg.size())) != hipSuccess ||
        (er = up(e->d_small, e->small_ids.data(), e->small_ids.size() * sizeof(int32_t))) != hipSuccess ||
        (er = up(e->d_big, e->big_ids.data(), e->big_ids.size() * sizeof(int32_t))) != hipSuccess ||
        (er = up(e->d_zitems, e->z_items.data(), e->z_items.size() * sizeof(BatchItem))) != hipSuccess)
        return hip_fail(er, "batch upload");
    for (auto& nd : e->nodes)
        if ((er = up(nd.d, nd.items.data(), nd.items.size() * sizeof(BatchItem))) != hipSuccess)
            return hip_fail(er, "batch upload");
    if ((er = hipMalloc((void**)&e->d_part, std::max<size_t>(e->total_part * QOPS_BATCH_REC, 1) * sizeof(double))) != hipSuccess ||
        (er = hipMalloc((void**)&e->d_out, std::max<size_t>(e->total_out, 1) * sizeof(double))) != hipSuccess)
        return hip_fail(er, "batch allocation");
    return QOPS_OK;
}

hipError_t enqueue(qops_batch_exec* e, hipStream_t s)
{
    hipError_t er = launch_batch_small(e->prec, e->d_small, (int)e->small_ids.size(), e->d_circs, e->d_ops, e->d_coef,
                                       e->d_out, e->lds_small, s);
    for (size_t k = 0; k < e->nodes.size() && er == hipSuccess; ++k) {
        const auto& nd = e->nodes[k];
        // register-tile items: 6144 one-wave work-groups (six per SIMD; as
        // many as the body's registers let reside: three at 148 VGPRs with
        // five register bits, six at 79-80 VGPRs with four) to hide the
        // global loads and lane exchanges
        if (nd.kind == 0)
            er = launch_batch_reg(e->prec, nd.R, nd.W, nd.d, (int)nd.items.size(), e->d_circs, e->d_hdrs, e->d_ops,
                                  e->d_coef, nd.pass, nd.lds, (e->grid * 12) >> nd.W, s);
        else
            er = launch_batch_pass(e->prec, nd.d, (int)nd.items.size(), e->d_circs, e->d_hdrs, e->d_ops, e->d_coef,
                                   nd.pass, nd.lds, e->grid, s);
    }
    if (er == hipSuccess)
        er = launch_batch_z(e->prec, e->d_zitems, (int)e->z_items.size(), e->d_big, (int)e->big_ids.size(), e->d_circs,
                            e->d_part, e->d_out, e->grid * 4, s);
    return er;
}

void release(qops_batch_exec* e)
{
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    void* ptrs[] = {e->d_circs, e->d_hdrs, e->d_ops, e->d_coef, e->d_small, e->d_big, e->d_zitems, e->d_part, e->d_out,
                    e->d_states};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& nd : e->nodes)
        if (nd.d) (void)hipFree(nd.d);
    if (e->own_stream && e->stream) (void)hipStreamDestroy(e->stream);
}

}  // namespace

extern "C" {

int32_t qops_batch_create(const qops_batch* b, qops_batch_exec** out)
{
    try {
        if (!b || !out || b->count < 1 || !b->n || !b->gates || !b->n_gates)
            return set_error(QOPS_INVALID_ARG, "bad batch description");
        if (b->precision != QOPS_C64 && b->precision != QOPS_C128) return set_error(QOPS_INVALID_ARG, "bad precision");
        *out = nullptr;
        std::unique_ptr<qops_batch_exec> e(new qops_batch_exec());
        e->prec = b->precision;
        e->count = b->count;
        const int lds_cap = b->precision == QOPS_C64 ? 13 : 12;
        e->small_max_n = b->small_max_n > 0 ? std::min(b->small_max_n, lds_cap) : lds_cap;
        e->tile_bits = b->tile_bits > 0 ? std::min(b->tile_bits, lds_cap) : lds_cap;
        if (e->tile_bits > e->small_max_n + 1) e->tile_bits = e->small_max_n + 1;
        if (e->tile_bits < 10) e->tile_bits = 10;
        e->fuse_k = b->max_fuse_k > 0 ? std::min(b->max_fuse_k, 6) : 1;
        int32_t rc = plan_all(e.get(), b);
        if (rc) return rc;
        rc = layout(e.get());
        if (rc) {
            release(e.get());
            return rc;
        }
        if (b->stream) {
            e->stream = reinterpret_cast<hipStream_t>(b->stream);
        } else {
            hipError_t er = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking);
            if (er != hipSuccess) {
                release(e.get());
                return hip_fail(er, "stream");
            }
            e->own_stream = true;
        }
        // one eager run (kernel attributes are set outside the capture), then
        // capture the whole batch as one graph
        hipError_t er = enqueue(e.get(), e->stream);
        if (er == hipSuccess) er = hipStreamSynchronize(e->stream);
        if (er != hipSuccess) {
            release(e.get());
            return hip_fail(er, "batch first run");
        }
        er = hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal);
        if (er == hipSuccess) {
            hipError_t el = enqueue(e.get(), e->stream);
            er = hipStreamEndCapture(e->stream, &e->graph);
            if (er == hipSuccess) er = el;
        }
        if (er == hipSuccess) er = hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0);
        if (er != hipSuccess) {
            release(e.get());
            return hip_fail(er, "graph capture");
        }
        *out = e.release();
        return QOPS_OK;
    } catch (...) {
        return set_error(QOPS_OUT_OF_MEMORY, "batch creation failed");
    }
}

int32_t qops_batch_launch(qops_batch_exec* e)
{
    if (!e) return set_error(QOPS_INVALID_ARG, "null batch");
    hipError_t er = hipGraphLaunch(e->exec, e->stream);
    if (er != hipSuccess) return hip_fail(er, "graph launch");
    return QOPS_OK;
}

int32_t qops_batch_results(qops_batch_exec* e, double* out_expz)
{
    if (!e || !out_expz) return set_error(QOPS_INVALID_ARG, "null argument");
    hipError_t er = hipMemcpyAsync(out_expz, e->d_out, e->total_out * sizeof(double), hipMemcpyDeviceToHost, e->stream);
    if (er == hipSuccess) er = hipStreamSynchronize(e->stream);
    if (er != hipSuccess) return hip_fail(er, "batch results");
    // the kernels reduce per physical bit; logical qubit q sits at l2p[q]
    std::vector<double> tmp;
    for (int i = 0; i < e->count; ++i) {
        const qops::Plan& p = e->plans[i];
        double* o = out_expz + e->circs[i].out0;
        bool ident = true;
        for (int q = 0; q < p.n; ++q) ident = ident && p.l2p_out[q] == q;
        if (ident) continue;
        tmp.assign(o, o + p.n);
        for (int q = 0; q < p.n; ++q) o[q] = tmp[p.l2p_out[q]];
    }
    return QOPS_OK;
}

int32_t qops_batch_time(qops_batch_exec* e, int32_t reps, double* seconds)
{
    if (!e || !seconds || reps < 1) return set_error(QOPS_INVALID_ARG, "bad arguments");
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return set_error(QOPS_HIP_ERROR, "event create");
    hipError_t er = hipEventRecord(a, e->stream);
    for (int r = 0; r < reps && er == hipSuccess; ++r) er = hipGraphLaunch(e->exec, e->stream);
    if (er == hipSuccess) er = hipEventRecord(b, e->stream);
    if (er == hipSuccess) er = hipEventSynchronize(b);
    float ms = 0;
    if (er == hipSuccess) er = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (er != hipSuccess) return hip_fail(er, "batch timing");
    *seconds = ms * 1e-3 / reps;
    e->last_seconds = *seconds;
    return QOPS_OK;
}

int32_t qops_batch_update(qops_batch_exec* e, const qops_gate* const* gates, const size_t* n_gates)
{
    try {
        if (!e || !gates || !n_gates) return set_error(QOPS_INVALID_ARG, "null argument");
        const size_t csz = e->prec == QOPS_C64 ? 4 : 8;
        std::vector<unsigned char> cimg;
        size_t total = 0;
        for (int i = 0; i < e->count; ++i) total = std::max(total, e->coef_base[i] + e->plans[i].coef.size());
        cimg.assign(std::max<size_t>(total, 1) * csz, 0);
        for (int i = 0; i < e->count; ++i) {
            qops::Plan& p = e->plans[i];
            const size_t before_ops = p.dops.size(), before_coef = p.coef.size();
            Err er = update_plan(p, gates[i], n_gates[i]);
            if (!er.ok()) return set_error(er.code, "circuit " + std::to_string(i) + ": " + er.msg);
            if (p.dops.size() != before_ops || p.coef.size() != before_coef)
                return set_error(QOPS_BAD_STATE, "circuit " + std::to_string(i) + ": new parameters change the plan");
            if (e->prec == QOPS_C64) cast_coef<float>(p.coef, cimg, e->coef_base[i]);
            else cast_coef<double>(p.coef, cimg, e->coef_base[i]);
        }
        hipError_t er = hipStreamSynchronize(e->stream);
        if (er == hipSuccess) er = hipMemcpy(e->d_coef, cimg.data(), total * csz, hipMemcpyHostToDevice);
        if (er != hipSuccess) return hip_fail(er, "batch update");
        return QOPS_OK;
    } catch (...) {
        return set_error(QOPS_OUT_OF_MEMORY, "batch update failed");
    }
}

int32_t qops_batch_info(const qops_batch_exec* e, qops_batch_stats* s)
{
    if (!e || !s) return set_error(QOPS_INVALID_ARG, "null argument");
    std::memset(s, 0, sizeof(*s));
    s->small_circuits = (int32_t)e->small_ids.size();
    s->tile_circuits = (int32_t)e->big_ids.size();
    s->graph_nodes = (int32_t)(e->nodes.size() + (e->small_ids.empty() ? 0 : 1) + (e->big_ids.empty() ? 0 : 2));
    s->small_max_n = e->small_max_n;
    s->tile_bits = e->tile_bits;
    s->max_fuse_k = e->fuse_k;
    s->outputs = (int64_t)e->total_out;
    s->state_bytes = (double)e->total_state_bytes;
    return QOPS_OK;
}

int32_t qops_batch_free(qops_batch_exec* e)
{
    if (!e) return QOPS_OK;
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    release(e);
    delete e;
    return QOPS_OK;
}

int32_t qops_batch_autotune(const qops_batch* b, const char* cache_path, int32_t* best_small_max_n,
                            int32_t* best_tile_bits, int32_t* best_fuse_k, double* best_seconds)
{
    if (!b || !best_small_max_n || !best_tile_bits || !best_fuse_k) return set_error(QOPS_INVALID_ARG, "null argument");
    // signature of the batch: size, precision, histogram of n
    int hist[27] = {0};
    for (int i = 0; i < b->count; ++i) hist[std::max(0, std::min(26, b->n[i]))]++;
    std::string sig = "p" + std::to_string(b->precision) + ":c" + std::to_string(b->count);
    for (int k = 0; k < 27; ++k)
        if (hist[k]) sig += ":" + std::to_string(k) + "x" + std::to_string(hist[k]);
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char line[4096];
            while (std::fgets(line, sizeof(line), f)) {
                char key[4000];
                int sm = 0, tb = 0, kf = 0;
                double sec = 0;
                if (std::sscanf(line, "%3999s %d %d %d %lf", key, &sm, &tb, &kf, &sec) == 5 && sig == key) {
                    std::fclose(f);
                    *best_small_max_n = sm;
                    *best_tile_bits = tb;
                    *best_fuse_k = kf;
                    if (best_seconds) *best_seconds = sec;
                    return QOPS_OK;
                }
            }
            std::fclose(f);
        }
    }
    const int cap = b->precision == QOPS_C64 ? 13 : 12;
    double best = -1;
    for (int kf = 1; kf <= 3; ++kf)
    for (int sm = 10; sm <= cap; ++sm)
        for (int tb = 11; tb <= cap; ++tb) {
            if (tb > sm + 1) continue;     // the executor would clamp it to sm + 1
            qops_batch bb = *b;
            bb.small_max_n = sm;
            bb.tile_bits = tb;
            bb.max_fuse_k = kf;
            qops_batch_exec* e = nullptr;
            int32_t rc = qops_batch_create(&bb, &e);
            if (rc) return rc;
            double sec = 0;
            rc = qops_batch_time(e, 1, &sec);
            if (!rc) rc = qops_batch_time(e, 3, &sec);
            qops_batch_free(e);
            if (rc) return rc;
            if (best < 0 || sec < best) {
                best = sec;
                *best_small_max_n = sm;
                *best_tile_bits = tb;
                *best_fuse_k = kf;
            }
        }
    if (best_seconds) *best_seconds = best;
    if (cache_path)
        if (FILE* f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "%s %d %d %d %.9g\n", sig.c_str(), *best_small_max_n, *best_tile_bits, *best_fuse_k, best);
            std::fclose(f);
        }
    return QOPS_OK;
}

}  // extern "C"
