// C ABI of libqops: handles, plan execution, layout, readout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qops.h"
#include "kernels.hpp"
#include "planner.hpp"
#include "runtime.hpp"

using namespace qops;

namespace qops {

thread_local std::string g_last_error;

int32_t set_error(int32_t code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

int32_t hip_fail(hipError_t e, const char* what)
{
    return set_error(e == hipErrorOutOfMemory ? QOPS_OUT_OF_MEMORY : QOPS_HIP_ERROR,
                     std::string(what) + ": " + hipGetErrorString(e));
}

size_t amp_size(int prec) { return prec == QOPS_C64 ? 8 : 16; }

// Uploads the plan's device program (once; again after an update).
int32_t upload_plan(Plan& p)
{
    if (!p.dirty) return QOPS_OK;
    auto realloc_copy = [&](void*& dptr, const void* src, size_t bytes) -> hipError_t {
        if (dptr) {
            hipError_t e = hipFree(dptr);
            dptr = nullptr;
            if (e != hipSuccess) return e;
        }
        if (bytes == 0) bytes = 64;
        hipError_t e = hipMalloc(&dptr, bytes);
        if (e != hipSuccess) return e;
        if (src) return hipMemcpy(dptr, src, bytes, hipMemcpyHostToDevice);
        return hipSuccess;
    };
    hipError_t e = realloc_copy(p.d_hdr, p.hdrs.empty() ? nullptr : p.hdrs.data(), p.hdrs.size() * sizeof(PassHdr));
    if (e != hipSuccess) return hip_fail(e, "plan upload");
    e = realloc_copy(p.d_ops, p.dops.empty() ? nullptr : p.dops.data(), p.dops.size() * sizeof(DevOp));
    if (e != hipSuccess) return hip_fail(e, "plan upload");
    if (p.prec == QOPS_C64) {
        std::vector<float> f(p.coef.begin(), p.coef.end());
        e = realloc_copy(p.d_coef, f.empty() ? nullptr : f.data(), f.size() * sizeof(float));
    } else {
        e = realloc_copy(p.d_coef, p.coef.empty() ? nullptr : p.coef.data(), p.coef.size() * sizeof(double));
    }
    if (e != hipSuccess) return hip_fail(e, "plan upload");
    p.dirty = false;
    return QOPS_OK;
}

void free_plan_device(Plan& p)
{
    if (p.d_hdr) (void)hipFree(p.d_hdr);
    if (p.d_ops) (void)hipFree(p.d_ops);
    if (p.d_coef) (void)hipFree(p.d_coef);
    p.d_hdr = p.d_ops = p.d_coef = nullptr;
    p.dirty = true;
}

// Launches one pass of a plan.
int32_t launch_pass(qops_sim* h, const Plan& p, const PassPlan& pp)
{
    hipError_t e = hipSuccess;
    const PassHdr* dh = reinterpret_cast<const PassHdr*>(p.d_hdr);
    const DevOp* dops = reinterpret_cast<const DevOp*>(p.d_ops);
    switch (pp.type) {
    case PASS_TILE_REG: {
        const uint64_t ntiles = 1ull << (p.n - pp.L);
        e = launch_tile_pass(p.prec, pp.R, pp.W, h->state, dh + pp.hdr, dops, p.d_coef, ntiles,
                             p.hdrs[pp.hdr].lds_bytes, h->grid_cap, h->stream);
        break;
    }
    case PASS_TILE_LDS: {
        const uint64_t ntiles = 1ull << (p.n - pp.L);
        const PassHdr& hh = p.hdrs[pp.hdr];
        const int hoist_k = hh.hoist >= 0 ? p.dops[hh.op0 + hh.hoist].a : 0;
        e = launch_tile_lds(p.prec, h->state, dh + pp.hdr, dops, p.d_coef, ntiles, pp.L, hh.lds_bytes, h->grid_cap,
                            hoist_k, h->stream);
        break;
    }
    case PASS_STATE_LDS:
        e = launch_state_lds(p.prec, h->state, p.n, dops + pp.op0, pp.nops, p.d_coef, h->stream);
        break;
    case PASS_SWEEP:
        e = launch_sweep(p.prec, h->state, p.n, &p.dops[pp.op0], p.d_coef, h->grid_cap, h->stream);
        break;
    case PASS_SWAP_BITS:
        e = launch_swap_bits(p.prec, h->state, p.n, std::min(pp.swap_a, pp.swap_b), std::max(pp.swap_a, pp.swap_b),
                             h->grid_cap, h->stream);
        break;
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QOPS_OK;
}

int32_t check_plan_matches(qops_sim* h, const Plan& p)
{
    if (p.n != h->n || p.prec != h->prec) return set_error(QOPS_BAD_STATE, "plan n/precision differ from the handle");
    for (int q = 0; q < h->n; ++q)
        if (p.l2p_in[q] != h->l2p[q]) return set_error(QOPS_BAD_STATE, "plan was built for another layout");
    return QOPS_OK;
}

int32_t run_plan(qops_sim* h, Plan& p)
{
    int32_t rc = check_plan_matches(h, p);
    if (rc) return rc;
    rc = upload_plan(p);
    if (rc) return rc;
    for (const PassPlan& pp : p.passes) {
        rc = launch_pass(h, p, pp);
        if (rc) return rc;
    }
    h->l2p = p.l2p_out;
    return QOPS_OK;
}

int32_t ensure_scratch(qops_sim* h, size_t doubles)
{
    if (h->scratch_doubles >= doubles) return QOPS_OK;
    if (h->scratch) {
        (void)hipFree(h->scratch);
        h->scratch = nullptr;
        h->scratch_doubles = 0;
    }
    hipError_t e = hipMalloc(&h->scratch, std::max<size_t>(doubles, 1024) * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "scratch allocation");
    h->scratch_doubles = std::max<size_t>(doubles, 1024);
    return QOPS_OK;
}

PlanParams params_from(const qops_plan_opts* o, int n, int prec)
{
    PlanParams par;
    // register tile passes: complex64 defaults to 4 register bits and no
    // wave bits (10-bit tiles, light enough for six waves per SIMD), which
    // measured 28-30 % faster than 13-bit tiles (5 register + 2 wave bits)
    // on gate-level circuits; LDS tile passes keep the largest tile
    par.R = 4;
    par.W = prec == QOPS_C64 ? 0 : 2;
    par.L_lds = prec == QOPS_C64 ? 13 : 12;
    par.state_lds_max_n = 12;
    if (!o) return par;
    par.mode = o->mode;
    par.swap_mode = o->swap_mode;
    if (o->tile_upper > 0) {
        // an explicit width: up to 5 (complex64) / 4 (complex128) register
        // bits, the rest wave bits
        par.R = prec == QOPS_C64 ? 5 : 4;
        par.W = std::max(0, o->tile_upper - par.R);
        if (o->tile_upper < par.R) {
            par.R = std::max(4, o->tile_upper);
            par.W = 0;
        }
        par.L_lds = std::min(6 + o->tile_upper, prec == QOPS_C64 ? 13 : 12);
    }
    par.max_fuse_k = o->max_fuse_k > 0 ? o->max_fuse_k : 1;
    par.fold = o->fold_rotations > 0 ? 1 : (o->fold_rotations < 0 ? -1 : 0);
    par.merge_blocks = o->merge_blocks > 0 ? 1 : (o->merge_blocks < 0 ? -1 : 0);
    par.remap = o->remap;
    par.use_mfma = o->use_mfma;
    par.check_unitary = o->check_unitary;
    (void)n;
    return par;
}

}  // namespace qops

namespace qops {

int32_t expect_zz(qops_sim* h, const int32_t* pairs, int32_t npairs, double* out)
{
    if (!h || (npairs > 0 && (!pairs || !out))) return set_error(QOPS_INVALID_ARG, "null argument");
    if (npairs < 0) return set_error(QOPS_INVALID_ARG, "npairs < 0");
    if (npairs == 0) return QOPS_OK;
    std::vector<int32_t> pa((size_t)npairs);
    std::vector<int32_t> pb((size_t)npairs);
    for (int i = 0; i < npairs; ++i) {
        const int a = pairs[2 * i];
        const int b = pairs[2 * i + 1];
        if (a < 0 || a >= h->n || b < 0 || b >= h->n) return set_error(QOPS_QUBIT_RANGE, "qubit out of range");
        pa[i] = h->l2p[a];
        pb[i] = h->l2p[b];
    }
    const size_t part = zz_scratch_doubles(h->n);
    int32_t rc = ensure_scratch(h, part + (size_t)npairs);
    if (rc) return rc;
    hipError_t e = launch_expect_zz(h->prec, h->state, h->n, pa.data(), pb.data(), npairs, h->scratch,
                                    h->scratch + part, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, h->scratch + part, (size_t)npairs * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "expect_zz");
    return QOPS_OK;
}

}  // namespace qops

// ===========================================================================
// C ABI
// ===========================================================================

#define QOPS_GUARD(expr)                                                          \
    try {                                                                         \
        expr;                                                                     \
    } catch (const std::bad_alloc&) {                                             \
        return set_error(QOPS_OUT_OF_MEMORY, "host allocation failed");           \
    } catch (...) {                                                               \
        return set_error(QOPS_INVALID_ARG, "internal error");                     \
    }

extern "C" {

const char* qops_last_error(void) { return g_last_error.c_str(); }

int32_t qops_version(void) { return 10000 * 0 + 100 * 3 + 0; }

int32_t qops_create(int32_t n, int32_t precision, void* dev_state, size_t bytes, void* stream, qops_sim** out)
{
    QOPS_GUARD({
        if (!out) return set_error(QOPS_INVALID_ARG, "out is null");
        *out = nullptr;
        if (n < 1 || n > QOPS_MAX_QUBITS) return set_error(QOPS_UNSUPPORTED, "n must be in [1, 34]");
        if (precision != QOPS_C64 && precision != QOPS_C128) return set_error(QOPS_INVALID_ARG, "bad precision");
        const size_t need = (size_t(1) << n) * amp_size(precision);
        std::unique_ptr<qops_sim> h(new qops_sim());
        h->n = n;
        h->prec = precision;
        h->bytes = need;
        h->stream = reinterpret_cast<hipStream_t>(stream);
        if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
        h->l2p.resize(n);
        for (int q = 0; q < n; ++q) h->l2p[q] = q;
        if (dev_state) {
            if (bytes < need) return set_error(QOPS_INVALID_ARG, "borrowed buffer is smaller than 2^n amplitudes");
            h->state = dev_state;
            h->owned = false;
        } else {
            hipError_t e = hipMalloc(&h->state, need);
            if (e != hipSuccess) return hip_fail(e, "state allocation");
            h->owned = true;
        }
        *out = h.release();
        return QOPS_OK;
    });
}

int32_t qops_destroy(qops_sim* h)
{
    if (!h) return QOPS_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->owned && h->state) (void)hipFree(h->state);
    if (h->scratch) (void)hipFree(h->scratch);
    for (auto& ev : h->events) (void)hipEventDestroy(ev);
    if (h->last_plan) {
        free_plan_device(*h->last_plan);
        delete h->last_plan;
    }
    delete h;
    return QOPS_OK;
}

int32_t qops_set_launch_limit(qops_sim* h, int32_t max_workgroups)
{
    if (!h) return set_error(QOPS_INVALID_ARG, "null handle");
    if (max_workgroups < 0) return set_error(QOPS_INVALID_ARG, "max_workgroups < 0");
    h->grid_cap = max_workgroups;
    return QOPS_OK;
}

int32_t qops_state_pointer(qops_sim* h, void** dev_ptr, size_t* bytes)
{
    if (!h || !dev_ptr) return set_error(QOPS_INVALID_ARG, "null argument");
    *dev_ptr = h->state;
    if (bytes) *bytes = h->bytes;
    return QOPS_OK;
}

int32_t qops_init_basis(qops_sim* h, uint64_t x)
{
    if (!h) return set_error(QOPS_INVALID_ARG, "null handle");
    if (h->n < 64 && x >= (1ull << h->n)) return set_error(QOPS_INVALID_ARG, "basis index out of range");
    for (int q = 0; q < h->n; ++q) h->l2p[q] = q;
    hipError_t e = launch_init_basis(h->prec, h->state, h->n, x, h->stream);
    if (e != hipSuccess) return hip_fail(e, "init_basis");
    return QOPS_OK;
}

int32_t qops_init_amplitudes(qops_sim* h, const void* host)
{
    if (!h || !host) return set_error(QOPS_INVALID_ARG, "null argument");
    for (int q = 0; q < h->n; ++q) h->l2p[q] = q;
    hipError_t e = hipMemcpyAsync(h->state, host, h->bytes, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "init_amplitudes");
    return QOPS_OK;
}

int32_t qops_plan_opts_default(qops_plan_opts* o)
{
    if (!o) return set_error(QOPS_INVALID_ARG, "null opts");
    std::memset(o, 0, sizeof(*o));
    o->mode = QOPS_PLAN_FUSED;
    o->swap_mode = QOPS_SWAP_VIRTUAL;
    o->use_mfma = 1;
    return QOPS_OK;
}

int32_t qops_plan_build(int32_t n, int32_t precision, const int32_t* l2p_in, const qops_gate* gates, size_t n_gates,
                        const qops_plan_opts* opts, qops_plan** out)
{
    QOPS_GUARD({
        if (!out) return set_error(QOPS_INVALID_ARG, "out is null");
        *out = nullptr;
        if (opts && (opts->mode < 0 || opts->mode > QOPS_PLAN_LEARNED))
            return set_error(QOPS_INVALID_ARG, "bad plan mode");
        if (opts && (opts->swap_mode < 0 || opts->swap_mode > 1)) return set_error(QOPS_INVALID_ARG, "bad swap mode");
        std::unique_ptr<qops_plan> p(new qops_plan());
        int32_t rc = build_priced_plan(n, precision, l2p_in, gates, n_gates, opts, p->p);
        if (rc) return rc;
        *out = p.release();
        return QOPS_OK;
    });
}

int32_t qops_plan_free(qops_plan* p)
{
    if (!p) return QOPS_OK;
    if (p->p.d_hdr || p->p.d_ops || p->p.d_coef) (void)hipDeviceSynchronize();
    free_plan_device(p->p);
    delete p;
    return QOPS_OK;
}

int32_t qops_plan_stats_get(const qops_plan* p, qops_plan_stats* s)
{
    if (!p || !s) return set_error(QOPS_INVALID_ARG, "null argument");
    std::memset(s, 0, sizeof(*s));
    const Plan& q = p->p;
    s->n_passes = (int32_t)q.passes.size();
    for (const PassPlan& pp : q.passes) {
        if (pp.type == PASS_TILE_REG || pp.type == PASS_TILE_LDS || pp.type == PASS_STATE_LDS) s->n_tile_passes++;
        if (pp.type == PASS_SWAP_BITS) s->n_permute_passes++;
        s->bytes_alg += pp.bytes_alg;
    }
    s->n_ops = (int32_t)q.lops.size();
    s->n_gates_in = (int32_t)q.gates.size();
    s->n_virtual_swaps = q.n_virtual_swaps;
    s->tile_upper = q.par.R + q.par.W;
    s->max_fuse_k = q.par.max_fuse_k;
    s->n_folded = q.n_folded;
    s->predicted_s = q.predicted_s;
    s->plan_seconds = q.plan_seconds;
    return QOPS_OK;
}

int32_t qops_plan_num_ops(const qops_plan* p, size_t* n)
{
    if (!p || !n) return set_error(QOPS_INVALID_ARG, "null argument");
    *n = p->p.lops.size();
    return QOPS_OK;
}

int32_t qops_plan_op(const qops_plan* p, size_t i, qops_op_info* info, double* mat)
{
    if (!p || !info) return set_error(QOPS_INVALID_ARG, "null argument");
    if (i >= p->p.lops.size()) return set_error(QOPS_INVALID_ARG, "op index out of range");
    const LOp& o = p->p.lops[i];
    std::memset(info, 0, sizeof(*info));
    info->kind = (int32_t)o.kind;
    info->k = o.k;
    for (int j = 0; j < o.k && j < 10; ++j) info->t[j] = o.t[j];
    info->cmask = o.cmask;
    info->n_merged = o.nmerged;
    info->pass = -1;
    for (size_t pi = 0; pi < p->p.passes.size(); ++pi)
        for (int li : p->p.passes[pi].lop)
            if ((size_t)li == i) info->pass = (int32_t)pi;
    if (mat)
        for (size_t j = 0; j < o.m.size(); ++j) {
            mat[2 * j] = o.m[j].real();
            mat[2 * j + 1] = o.m[j].imag();
        }
    return QOPS_OK;
}

int32_t qops_plan_pass_info(const qops_plan* p, size_t i, qops_pass_info* info)
{
    if (!p || !info) return set_error(QOPS_INVALID_ARG, "null argument");
    if (i >= p->p.passes.size()) return set_error(QOPS_INVALID_ARG, "pass index out of range");
    const PassPlan& pp = p->p.passes[i];
    std::memset(info, 0, sizeof(*info));
    info->type = (int32_t)pp.type;
    info->tile_bits = pp.L;
    info->n_upper = (int32_t)pp.up.size();
    for (size_t u = 0; u < pp.up.size() && u < 8; ++u) info->upper[u] = pp.up[u];
    info->n_ops = (int32_t)pp.lop.size();
    info->n_remaps = pp.n_remaps;
    info->n_mfma = pp.n_mfma;
    info->bytes_alg = pp.bytes_alg;
    info->flops = pp.flops;
    return QOPS_OK;
}

int32_t qops_plan_final_layout(const qops_plan* p, int32_t* l2p)
{
    if (!p || !l2p) return set_error(QOPS_INVALID_ARG, "null argument");
    for (int q = 0; q < p->p.n; ++q) l2p[q] = p->p.l2p_out[q];
    return QOPS_OK;
}

int32_t qops_run_plan(qops_sim* h, const qops_plan* p)
{
    QOPS_GUARD({
        if (!h || !p) return set_error(QOPS_INVALID_ARG, "null argument");
        return run_plan(h, const_cast<qops_plan*>(p)->p);
    });
}

int32_t qops_plan_update(qops_plan* p, const qops_gate* gates, size_t n_gates)
{
    QOPS_GUARD({
        if (!p) return set_error(QOPS_INVALID_ARG, "null plan");
        (void)hipDeviceSynchronize();
        Err e = update_plan(p->p, gates, n_gates);
        if (!e.ok()) return set_error(e.code, e.msg);
        return QOPS_OK;
    });
}

int32_t qops_apply(qops_sim* h, const qops_gate* gates, size_t n_gates, const qops_plan_opts* opts)
{
    QOPS_GUARD({
        if (!h) return set_error(QOPS_INVALID_ARG, "null handle");
        std::unique_ptr<Plan> p(new Plan());
        int32_t rc = build_priced_plan(h->n, h->prec, h->l2p.data(), gates, n_gates, opts, *p);
        if (rc) return rc;
        if (h->last_plan) {
            (void)hipStreamSynchronize(h->stream);
            free_plan_device(*h->last_plan);
            delete h->last_plan;
            h->last_plan = nullptr;
        }
        rc = run_plan(h, *p);
        h->last_plan = p.release();
        return rc;
    });
}

int32_t qops_swap(qops_sim* h, int32_t a, int32_t b, int32_t mode)
{
    if (!h) return set_error(QOPS_INVALID_ARG, "null handle");
    if (a < 0 || a >= h->n || b < 0 || b >= h->n) return set_error(QOPS_QUBIT_RANGE, "qubit out of range");
    if (a == b) return set_error(QOPS_DUPLICATE_QUBIT, "swap of a qubit with itself");
    if (mode == QOPS_SWAP_VIRTUAL) {
        std::swap(h->l2p[a], h->l2p[b]);
        return QOPS_OK;
    }
    if (mode != QOPS_SWAP_PHYSICAL) return set_error(QOPS_INVALID_ARG, "bad swap mode");
    const int pa = h->l2p[a], pb = h->l2p[b];
    hipError_t e = launch_swap_bits(h->prec, h->state, h->n, std::min(pa, pb), std::max(pa, pb), h->grid_cap, h->stream);
    if (e != hipSuccess) return hip_fail(e, "swap");
    return QOPS_OK;
}

int32_t qops_get_layout(qops_sim* h, int32_t* l2p)
{
    if (!h || !l2p) return set_error(QOPS_INVALID_ARG, "null argument");
    for (int q = 0; q < h->n; ++q) l2p[q] = h->l2p[q];
    return QOPS_OK;
}

int32_t qops_set_layout(qops_sim* h, const int32_t* l2p)
{
    if (!h || !l2p) return set_error(QOPS_INVALID_ARG, "null argument");
    const int n = h->n;
    uint64_t seen = 0;
    for (int q = 0; q < n; ++q) {
        if (l2p[q] < 0 || l2p[q] >= n || (seen & (1ull << l2p[q])))
            return set_error(QOPS_INVALID_ARG, "l2p is not a permutation");
        seen |= 1ull << l2p[q];
    }
    // Transposition sort: move logical qubit q to physical l2p[q] one bit
    // exchange at a time (at most n-1 passes).
    std::vector<int> cur = h->l2p;
    std::vector<int> p2l(n);
    for (int q = 0; q < n; ++q) p2l[cur[q]] = q;
    for (int q = 0; q < n; ++q) {
        const int want = l2p[q], have = cur[q];
        if (want == have) continue;
        hipError_t e = launch_swap_bits(h->prec, h->state, n, std::min(want, have), std::max(want, have), h->grid_cap,
                                        h->stream);
        if (e != hipSuccess) return hip_fail(e, "set_layout");
        const int other = p2l[want];
        cur[other] = have;
        p2l[have] = other;
        cur[q] = want;
        p2l[want] = q;
    }
    h->l2p = cur;
    return QOPS_OK;
}

int32_t qops_read_state(qops_sim* h, void* host, int32_t order)
{
    QOPS_GUARD({
        if (!h || !host) return set_error(QOPS_INVALID_ARG, "null argument");
        const size_t asz = amp_size(h->prec);
        bool identity = true;
        for (int q = 0; q < h->n; ++q) identity = identity && h->l2p[q] == q;
        hipError_t e;
        if (order == QOPS_ORDER_PHYSICAL || identity) {
            e = hipMemcpyAsync(host, h->state, h->bytes, hipMemcpyDeviceToHost, h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return hip_fail(e, "read_state");
            return QOPS_OK;
        }
        if (order != QOPS_ORDER_LOGICAL) return set_error(QOPS_INVALID_ARG, "bad order");
        // gather logical chunks on the device, then copy each chunk
        const uint64_t N = 1ull << h->n;
        const uint64_t chunk = std::min<uint64_t>(N, 1ull << 24);
        int32_t rc = ensure_scratch(h, (chunk * asz + 7) / 8);
        if (rc) return rc;
        for (uint64_t x0 = 0; x0 < N; x0 += chunk) {
            e = launch_gather_logical(h->prec, h->state, h->n, h->l2p.data(), x0, chunk, h->scratch, h->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(static_cast<char*>(host) + x0 * asz, h->scratch, chunk * asz, hipMemcpyDeviceToHost,
                                   h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return hip_fail(e, "read_state");
        }
        return QOPS_OK;
    });
}

static int32_t zsum(qops_sim* h, std::vector<double>& out)
{
    const int n = h->n;
    const size_t part = zsum_scratch_doubles(n);
    int32_t rc = ensure_scratch(h, part + n + 1);
    if (rc) return rc;
    double* d_out = h->scratch + part;
    hipError_t e = launch_zsum(h->prec, h->state, n, h->scratch, d_out, h->stream);
    out.assign(n + 1, 0.0);
    if (e == hipSuccess) e = hipMemcpyAsync(out.data(), d_out, (n + 1) * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "reduction");
    return QOPS_OK;
}

int32_t qops_norm(qops_sim* h, double* out)
{
    QOPS_GUARD({
        if (!h || !out) return set_error(QOPS_INVALID_ARG, "null argument");
        std::vector<double> v;
        int32_t rc = zsum(h, v);
        if (rc) return rc;
        *out = v[0];
        return QOPS_OK;
    });
}

int32_t qops_expect_z(qops_sim* h, double* out)
{
    QOPS_GUARD({
        if (!h || !out) return set_error(QOPS_INVALID_ARG, "null argument");
        std::vector<double> v;
        int32_t rc = zsum(h, v);
        if (rc) return rc;
        for (int q = 0; q < h->n; ++q) out[q] = v[0] - 2.0 * v[1 + h->l2p[q]];
        return QOPS_OK;
    });
}

int32_t qops_expect_zz(qops_sim* h, const int32_t* pairs, int32_t npairs, double* out)
{
    QOPS_GUARD(return qops::expect_zz(h, pairs, npairs, out));
}

int32_t qops_probabilities(qops_sim* h, const int32_t* qubits, int32_t m, double* out)
{
    QOPS_GUARD({
        if (!h || !qubits || !out) return set_error(QOPS_INVALID_ARG, "null argument");
        if (m < 1 || m > h->n) return set_error(QOPS_INVALID_ARG, "m must be in [1, n]");
        if (m > 30) return set_error(QOPS_UNSUPPORTED, "more than 30 marginal qubits");
        std::vector<int> pos(m);
        uint64_t seen = 0;
        for (int j = 0; j < m; ++j) {
            if (qubits[j] < 0 || qubits[j] >= h->n) return set_error(QOPS_QUBIT_RANGE, "qubit out of range");
            if (seen & (1ull << qubits[j])) return set_error(QOPS_DUPLICATE_QUBIT, "qubit listed twice");
            seen |= 1ull << qubits[j];
            pos[j] = h->l2p[qubits[j]];
        }
        const size_t ny = size_t(1) << m;
        const size_t part = probs_scratch_doubles(h->n, m, pos.data());
        int32_t rc = ensure_scratch(h, part + ny);
        if (rc) return rc;
        double* d_out = h->scratch + part;
        hipError_t e = launch_probs(h->prec, h->state, h->n, m, pos.data(), h->scratch, d_out, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, ny * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "probabilities");
        return QOPS_OK;
    });
}

int32_t qops_synchronize(qops_sim* h)
{
    if (!h) return set_error(QOPS_INVALID_ARG, "null handle");
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "synchronize");
    return QOPS_OK;
}

}  // extern "C"
