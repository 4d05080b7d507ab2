// Host-memory state tier (paper Sec. II-B, the storage-based simulator's
// "file segment"): the top g physical index bits of the state select one of
// 2^g segments kept in pinned host memory; the device works on groups of
// segments at a time.  A gate whose non-diagonal target is a global (segment)
// bit needs the segments that differ in that bit on the device together, so
// the planner cuts the circuit into stages: every stage streams the whole
// state through the device once, in groups that hold the stage's active
// global bits as their top local bits, while the inactive global bits are
// fixed per group (controls on them select the group, diagonal phases on them
// become constants).  The profile-guided virtual swap of Sec. III-D decides
// which qubits live in the global bits: the initial placement puts the
// qubits that non-diagonal gates touch least (the gate counters of the
// profile) into the segment bits, and when a stage has to activate a global
// bit it exchanges it, inside the device group, with the local bit whose
// qubit is needed again latest, so that later gates on the hot qubit stay
// local.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/qops.h"
#include "kernels.hpp"
#include "planner.hpp"
#include "runtime.hpp"

using namespace qops;

namespace qops {

struct TierGroup {
    uint64_t inactive_val = 0;          // values of the inactive global bits (as a physical mask)
    std::vector<uint64_t> segments;     // host segment of device slot part j (2^m of them)
    Plan plan;                          // the group's operations on n_loc + m bits
};

struct TierStage {
    std::vector<int> active;            // active global bits (physical), in device order
    std::vector<TierGroup> groups;
    int n_ops = 0;                      // operations of the stage (before specialisation)
    int n_exchanges = 0;                // global<->local exchanges it performs
};

struct TierProgram {
    std::vector<TierStage> stages;
    std::vector<int> l2p_out;
    int n_virtual_swaps = 0;
    int n_exchanges = 0;
    double plan_seconds = 0;
};

// First placement of a basis state: the g logical qubits that non-diagonal
// gates touch least (ties: first touched latest) take the segment bits.
static std::vector<int> placement_from_counts(int n, int g, const qops_gate* gates, size_t ng)
{
    std::vector<long> hits(n, 0);
    std::vector<long> first(n, (long)ng);
    for (size_t i = 0; i < ng; ++i) {
        const qops_gate& x = gates[i];
        if (diag_kind(x.kind) || (x.kind == QOPS_SWAP && x.n_ctrl == 0)) continue;
        const int k = x.kind == QOPS_DENSE ? x.k : gate_arity(x.kind);
        for (int j = 0; j < k; ++j) {
            if (x.kind == QOPS_CX && j == 0) continue;   // the control of CX is diagonal
            hits[x.q[j]]++;
            first[x.q[j]] = std::min(first[x.q[j]], (long)i);
        }
    }
    std::vector<int> order(n);
    for (int q = 0; q < n; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (hits[a] != hits[b]) return hits[a] < hits[b];
        return first[a] > first[b];
    });
    std::vector<int> l2p(n, -1);
    std::vector<bool> global(n, false);
    for (int i = 0; i < g; ++i) global[order[i]] = true;
    // global qubits keep their relative order in the top bits, local ones in
    // the low bits
    int nl = 0, ngl = n - g;
    for (int q = 0; q < n; ++q) {
        if (global[q]) l2p[q] = ngl++;
        else l2p[q] = nl++;
    }
    return l2p;
}

// Specialises an operation to a group: bits in `inactive` are fixed to the
// group's values `val`; the others are renumbered by `pos` (physical bit ->
// group bit).  Returns false if the operation does nothing in this group.
static bool specialise(const LOp& o, uint64_t inactive, uint64_t val, const std::vector<int>& pos, LOp& out)
{
    out = o;
    if (o.kind == LOp::DIAG) {
        // keep the table entries whose inactive bits equal the group's values
        std::vector<int> keep;
        uint64_t fixed_idx = 0;
        for (int j = 0; j < o.k; ++j) {
            const uint64_t b = 1ull << o.t[j];
            if (inactive & b) {
                if (val & b) fixed_idx |= 1ull << j;
            } else {
                keep.push_back(j);
            }
        }
        const int k2 = (int)keep.size();
        std::vector<cd> tab((size_t)1 << k2);
        for (size_t i = 0; i < tab.size(); ++i) {
            uint64_t idx = fixed_idx;
            for (int j = 0; j < k2; ++j)
                if (i & (1ull << j)) idx |= 1ull << keep[j];
            tab[i] = o.m[idx];
        }
        if (k2 == 0) {
            // a constant phase on the whole group: a table over group bit 0
            if (tab[0] == cd(1, 0)) return false;
            out.k = 1;
            out.t[0] = 0;
            out.m = {tab[0], tab[0]};
            out.cphase = false;
            return true;
        }
        bool ident = true;
        for (const cd& v : tab) ident = ident && v == cd(1, 0);
        if (ident) return false;
        out.k = k2;
        for (int j = 0; j < k2; ++j) out.t[j] = pos[o.t[keep[j]]];
        out.m.swap(tab);
        out.cphase = true;
        for (size_t i = 0; i + 1 < out.m.size(); ++i) out.cphase = out.cphase && out.m[i] == cd(1, 0);
        return true;
    }
    // controls on inactive global bits select the group
    const uint64_t cin = o.cmask & inactive;
    if ((val & cin) != cin) return false;
    uint64_t cm = 0;
    for (int b = 0; b < 64; ++b)
        if (((o.cmask & ~inactive) >> b) & 1ull) cm |= 1ull << pos[b];
    out.cmask = cm;
    for (int j = 0; j < o.k; ++j) out.t[j] = pos[o.t[j]];
    return true;
}

// Cuts lowered operations into stages (see the file comment).  `ops` are on
// physical bits of the n-bit state as lowered from the layout the run starts
// in; exchanges inserted here renumber the later operations.
static Err make_program(int n, int prec, int g, int amax, std::vector<LOp>& ops, bool exchange,
                        const PlanParams& par, bool build_plans, TierProgram& prog, std::vector<int>& perm_out)
{
    const int nloc = n - g;
    const uint64_t gmask = ((n >= 64 ? ~0ull : (1ull << n) - 1)) & ~((1ull << nloc) - 1);
    // perm[x]: the bit that data lowered at physical bit x occupies now
    std::vector<int> perm(n), inv(n);
    for (int b = 0; b < n; ++b) perm[b] = inv[b] = b;
    // next non-diagonal use of each lowered bit after op i
    std::vector<std::vector<int>> uses(n);
    for (size_t i = 0; i < ops.size(); ++i) {
        const uint64_t tm = ops[i].tmask();
        for (int b = 0; b < n; ++b)
            if ((tm >> b) & 1ull) uses[b].push_back((int)i);
    }
    auto next_use = [&](int lowered_bit, int i) {
        const std::vector<int>& u = uses[lowered_bit];
        auto it = std::upper_bound(u.begin(), u.end(), i);
        return it == u.end() ? (int)ops.size() + 1 : *it;
    };
    auto mapped = [&](const LOp& o) {
        LOp m = o;
        for (int j = 0; j < o.k; ++j) m.t[j] = perm[o.t[j]];
        uint64_t cm = 0;
        for (int b = 0; b < n; ++b)
            if ((o.cmask >> b) & 1ull) cm |= 1ull << perm[b];
        m.cmask = cm;
        return m;
    };
    struct Raw {
        std::vector<int> active;
        std::vector<LOp> ops;
        int n_ex = 0;
    };
    std::vector<Raw> raw;
    raw.emplace_back();
    auto popc = [](uint64_t v) { return __builtin_popcountll(v); };
    uint64_t A = 0;
    for (size_t i = 0; i < ops.size(); ++i) {
        LOp o = mapped(ops[i]);
        const uint64_t need = o.tmask() & gmask;
        if (popc(need) > amax)
            return Err{QOPS_UNSUPPORTED, "a gate targets more global bits than a device group holds"};
        if ((need & ~A) != 0) {
            if (popc(A | need) > amax) {
                raw.emplace_back();
                A = 0;
            }
            for (int b = nloc; b < n; ++b) {
                if (!((need >> b) & 1ull) || ((A >> b) & 1ull)) continue;
                A |= 1ull << b;
                raw.back().active.push_back(b);
                if (!exchange) continue;
                // exchange global bit b with the local bit whose data is
                // needed again latest (never, at best); the op's own bits are
                // excluded
                const uint64_t own = o.touch();
                int best = -1, best_use = -1;
                for (int c = 0; c < nloc; ++c) {
                    if ((own >> c) & 1ull) continue;
                    const int u = next_use(inv[c], (int)i);
                    if (u > best_use) {
                        best_use = u;
                        best = c;
                    }
                }
                if (best < 0) continue;
                LOp sw;
                sw.kind = LOp::PSWAP;
                sw.k = 2;
                sw.t[0] = best;
                sw.t[1] = b;
                raw.back().ops.push_back(sw);
                raw.back().n_ex++;
                prog.n_exchanges++;
                const int xb = inv[b], xc = inv[best];
                perm[xb] = best;
                perm[xc] = b;
                inv[best] = xb;
                inv[b] = xc;
                o = mapped(ops[i]);
            }
        }
        raw.back().ops.push_back(o);
    }
    perm_out = perm;
    // groups of every stage
    prog.stages.clear();
    for (Raw& r : raw) {
        if (r.ops.empty()) continue;
        TierStage st;
        st.active = r.active;
        std::sort(st.active.begin(), st.active.end());
        st.n_ops = (int)r.ops.size();
        st.n_exchanges = r.n_ex;
        const int m = (int)st.active.size();
        uint64_t amask = 0;
        for (int b : st.active) amask |= 1ull << b;
        const uint64_t inactive = gmask & ~amask;
        std::vector<int> ibits;
        for (int b = nloc; b < n; ++b)
            if ((inactive >> b) & 1ull) ibits.push_back(b);
        std::vector<int> pos(64, -1);
        for (int b = 0; b < nloc; ++b) pos[b] = b;
        for (int j = 0; j < m; ++j) pos[st.active[j]] = nloc + j;
        const uint64_t ngroups = 1ull << ibits.size();
        for (uint64_t v = 0; v < ngroups; ++v) {
            TierGroup tg;
            uint64_t val = 0;
            for (size_t j = 0; j < ibits.size(); ++j)
                if ((v >> j) & 1ull) val |= 1ull << ibits[j];
            tg.inactive_val = val;
            for (uint64_t a = 0; a < (1ull << m); ++a) {
                uint64_t phys = val;
                for (int j = 0; j < m; ++j)
                    if ((a >> j) & 1ull) phys |= 1ull << st.active[j];
                tg.segments.push_back(phys >> nloc);
            }
            if (build_plans) {
                std::vector<LOp> gops;
                for (const LOp& o : r.ops) {
                    LOp so;
                    if (specialise(o, inactive, val, pos, so)) gops.push_back(so);
                }
                Err e = plan_from_lops(nloc + m, prec, gops, par, tg.plan);
                if (!e.ok()) return e;
            }
            st.groups.push_back(std::move(tg));
        }
        prog.stages.push_back(std::move(st));
    }
    return Err{};
}

// Lowers and stages a gate list from layout l2p (updated to the layout the
// program leaves).
static Err plan_tier(int n, int prec, int g, int amax, std::vector<int>& l2p, const qops_gate* gates, size_t ng,
                     bool exchange, const PlanParams& par, bool build_plans, TierProgram& prog)
{
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<LOp> ops;
    int nvirt = 0;
    Err e = lower_gates(n, gates, ng, par.swap_mode, l2p, ops, nvirt);
    if (!e.ok()) return e;
    std::vector<int> perm;
    e = make_program(n, prec, g, amax, ops, exchange, par, build_plans, prog, perm);
    if (!e.ok()) return e;
    for (int q = 0; q < n; ++q) l2p[q] = perm[l2p[q]];
    prog.l2p_out = l2p;
    prog.n_virtual_swaps = nvirt;
    prog.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return Err{};
}

}  // namespace qops

struct qops_tier {
    int n = 0, prec = 0, g = 0, amax = 1;
    int nloc = 0;
    std::vector<char*> seg;                // host segment s (2^(n-g) amplitudes each)
    bool host_owned = false;               // segments allocated by the library, one pinned block each
    size_t bytes = 0;
    void* dev[2] = {nullptr, nullptr};
    size_t slot_bytes = 0;
    hipStream_t stream = nullptr;          // compute stream (the caller's)
    hipStream_t copy_in = nullptr, copy_out = nullptr;
    hipEvent_t loaded[2] = {}, computed[2] = {}, stored[2] = {};
    std::vector<int> l2p;
    bool basis = false;                    // the state is a basis state set by init_basis
    uint64_t basis_x = 0;
    double* scratch = nullptr;             // readout partial sums
    size_t scratch_doubles = 0;
};

namespace {

// Zeroes a large host buffer with several threads (a 128 GiB state would
// take tens of seconds on one core).
void parallel_zero(void* p, size_t bytes)
{
    const size_t chunk = size_t(1) << 28;
    if (bytes <= chunk) {
        std::memset(p, 0, bytes);
        return;
    }
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned i = 0; i < nt; ++i)
        th.emplace_back([=]() {
            for (size_t o = (size_t)i * chunk; o < bytes; o += (size_t)nt * chunk)
                std::memset(static_cast<char*>(p) + o, 0, std::min(chunk, bytes - o));
        });
    for (auto& x : th) x.join();
}

uint64_t basis_phys(const qops_tier* t)
{
    uint64_t phys = 0;
    for (int q = 0; q < t->n; ++q)
        if ((t->basis_x >> q) & 1ull) phys |= 1ull << t->l2p[q];
    return phys;
}

size_t seg_bytes_of(const qops_tier* t) { return ((size_t)1 << t->nloc) * amp_size(t->prec); }

char* amp_ptr(qops_tier* t, uint64_t phys)
{
    return t->seg[phys >> t->nloc] + (phys & ((1ull << t->nloc) - 1ull)) * amp_size(t->prec);
}

void put_one(qops_tier* t, uint64_t phys, bool one)
{
    char* p = amp_ptr(t, phys);
    if (t->prec == QOPS_C64) {
        const float v[2] = {one ? 1.f : 0.f, 0.f};
        std::memcpy(p, v, sizeof(v));
    } else {
        const double v[2] = {one ? 1.0 : 0.0, 0.0};
        std::memcpy(p, v, sizeof(v));
    }
}

int32_t tier_copy_basis(qops_tier* t)
{
    const uint64_t phys = basis_phys(t);
    for (char* sp : t->seg) parallel_zero(sp, seg_bytes_of(t));
    char* p = amp_ptr(t, phys);
    if (t->prec == QOPS_C64) {
        const float one[2] = {1.f, 0.f};
        std::memcpy(p, one, sizeof(one));
    } else {
        const double one[2] = {1.0, 0.0};
        std::memcpy(p, one, sizeof(one));
    }
    return QOPS_OK;
}

// One group: H2D of its segments, its plan, D2H back, pipelined over the two
// device slots (item index `item`).  `after_prev_stage` makes the loads wait
// for every store of the previous stage.
int32_t tier_group(qops_tier* t, TierGroup& grp, int m, size_t item, bool after_prev_stage, qops_sim& sim)
{
    const int slot = (int)(item & 1);
    const size_t seg_bytes = ((size_t)1 << t->nloc) * amp_size(t->prec);
    hipError_t e = hipSuccess;
    if (item >= 2) e = hipStreamWaitEvent(t->copy_in, t->stored[slot], 0);
    if (e == hipSuccess && after_prev_stage && item >= 1) e = hipStreamWaitEvent(t->copy_in, t->stored[slot ^ 1], 0);
    for (size_t j = 0; j < grp.segments.size() && e == hipSuccess; ++j)
        e = hipMemcpyAsync(static_cast<char*>(t->dev[slot]) + j * seg_bytes,
                           t->seg[grp.segments[j]], seg_bytes,
                           hipMemcpyHostToDevice, t->copy_in);
    if (e == hipSuccess) e = hipEventRecord(t->loaded[slot], t->copy_in);
    if (e == hipSuccess) e = hipStreamWaitEvent(t->stream, t->loaded[slot], 0);
    if (e != hipSuccess) return hip_fail(e, "tier load");
    sim.n = t->nloc + m;
    sim.state = t->dev[slot];
    sim.bytes = ((size_t)1 << sim.n) * amp_size(t->prec);
    sim.l2p.resize(sim.n);
    for (int q = 0; q < sim.n; ++q) sim.l2p[q] = q;
    int32_t rc = run_plan(&sim, grp.plan);
    if (rc) return rc;
    e = hipEventRecord(t->computed[slot], t->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(t->copy_out, t->computed[slot], 0);
    for (size_t j = 0; j < grp.segments.size() && e == hipSuccess; ++j)
        e = hipMemcpyAsync(t->seg[grp.segments[j]],
                           static_cast<char*>(t->dev[slot]) + j * seg_bytes, seg_bytes, hipMemcpyDeviceToHost,
                           t->copy_out);
    if (e == hipSuccess) e = hipEventRecord(t->stored[slot], t->copy_out);
    if (e != hipSuccess) return hip_fail(e, "tier store");
    return QOPS_OK;
}

void fill_stats(const TierProgram& prog, const qops_tier* t, qops_tier_stats* st)
{
    if (!st) return;
    std::memset(st, 0, sizeof(*st));
    st->stages = (int32_t)prog.stages.size();
    st->exchanges = prog.n_exchanges;
    st->virtual_swaps = prog.n_virtual_swaps;
    st->plan_seconds = prog.plan_seconds;
    double seg = t ? (double)((size_t)1 << t->nloc) * (double)amp_size(t->prec) : 0.0;
    for (const TierStage& s : prog.stages) {
        st->groups += (int32_t)s.groups.size();
        for (const TierGroup& gr : s.groups) {
            st->h2d_bytes += seg * (double)gr.segments.size();
            st->gpu_passes += (int32_t)gr.plan.passes.size();
        }
    }
    st->d2h_bytes = st->h2d_bytes;
}

}  // namespace

extern "C" {

int32_t qops_tier_opts_default(qops_tier_opts* o)
{
    if (!o) return set_error(QOPS_INVALID_ARG, "null opts");
    std::memset(o, 0, sizeof(*o));
    o->remap = 1;
    return qops_plan_opts_default(&o->plan);
}

int32_t qops_tier_create(int32_t n, int32_t precision, int32_t global_bits, int32_t max_active, void* host_state,
                         size_t bytes, void* stream, qops_tier** out)
{
    try {
        if (!out) return set_error(QOPS_INVALID_ARG, "out is null");
        *out = nullptr;
        if (n < 2 || n > QOPS_MAX_QUBITS) return set_error(QOPS_UNSUPPORTED, "n must be in [2, 34]");
        if (precision != QOPS_C64 && precision != QOPS_C128) return set_error(QOPS_INVALID_ARG, "bad precision");
        if (global_bits < 1 || global_bits > 8 || global_bits >= n)
            return set_error(QOPS_UNSUPPORTED, "global_bits must be in [1, min(8, n-1)]");
        if (max_active < 1 || max_active > global_bits)
            return set_error(QOPS_INVALID_ARG, "max_active must be in [1, global_bits]");
        std::unique_ptr<qops_tier> t(new qops_tier());
        t->n = n;
        t->prec = precision;
        t->g = global_bits;
        t->amax = max_active;
        t->nloc = n - global_bits;
        t->bytes = ((size_t)1 << n) * amp_size(precision);
        t->stream = reinterpret_cast<hipStream_t>(stream);
        t->l2p.resize(n);
        for (int q = 0; q < n; ++q) t->l2p[q] = q;
        hipError_t e;
        const size_t segb = ((size_t)1 << t->nloc) * amp_size(precision);
        t->seg.assign((size_t)1 << global_bits, nullptr);
        auto cleanup = [&]() {
            for (int s = 0; s < 2; ++s) {
                if (t->loaded[s]) (void)hipEventDestroy(t->loaded[s]);
                if (t->computed[s]) (void)hipEventDestroy(t->computed[s]);
                if (t->stored[s]) (void)hipEventDestroy(t->stored[s]);
            }
            if (t->copy_in) (void)hipStreamDestroy(t->copy_in);
            if (t->copy_out) (void)hipStreamDestroy(t->copy_out);
            for (void* d : t->dev)
                if (d) (void)hipFree(d);
            if (t->host_owned)
                for (char* sp : t->seg)
                    if (sp) (void)hipHostFree(sp);
        };
        if (host_state) {
            if (bytes < t->bytes) return set_error(QOPS_INVALID_ARG, "host buffer is smaller than 2^n amplitudes");
            for (size_t sgi = 0; sgi < t->seg.size(); ++sgi) t->seg[sgi] = static_cast<char*>(host_state) + sgi * segb;
        } else {
            t->host_owned = true;
            for (size_t sgi = 0; sgi < t->seg.size(); ++sgi) {
                void* sp = nullptr;
                e = hipHostMalloc(&sp, segb, hipHostMallocDefault);
                if (e != hipSuccess) {
                    cleanup();
                    return hip_fail(e, "pinned host segment");
                }
                t->seg[sgi] = static_cast<char*>(sp);
            }
        }
        t->slot_bytes = ((size_t)1 << (t->nloc + max_active)) * amp_size(precision);
        for (int s = 0; s < 2; ++s) {
            e = hipMalloc(&t->dev[s], t->slot_bytes);
            if (e != hipSuccess) {
                cleanup();
                return hip_fail(e, "device group slots");
            }
        }
        e = hipStreamCreateWithFlags(&t->copy_in, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&t->copy_out, hipStreamNonBlocking);
        for (int s = 0; s < 2 && e == hipSuccess; ++s) {
            e = hipEventCreateWithFlags(&t->loaded[s], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&t->computed[s], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&t->stored[s], hipEventDisableTiming);
        }
        if (e != hipSuccess) {
            cleanup();
            return hip_fail(e, "tier streams");
        }
        *out = t.release();
        return QOPS_OK;
    } catch (...) {
        return set_error(QOPS_OUT_OF_MEMORY, "host allocation failed");
    }
}

int32_t qops_tier_destroy(qops_tier* t)
{
    if (!t) return QOPS_OK;
    (void)hipStreamSynchronize(t->stream);
    if (t->copy_in) (void)hipStreamSynchronize(t->copy_in);
    if (t->copy_out) (void)hipStreamSynchronize(t->copy_out);
    for (int s = 0; s < 2; ++s) {
        if (t->loaded[s]) (void)hipEventDestroy(t->loaded[s]);
        if (t->computed[s]) (void)hipEventDestroy(t->computed[s]);
        if (t->stored[s]) (void)hipEventDestroy(t->stored[s]);
        if (t->dev[s]) (void)hipFree(t->dev[s]);
    }
    if (t->copy_in) (void)hipStreamDestroy(t->copy_in);
    if (t->copy_out) (void)hipStreamDestroy(t->copy_out);
    if (t->scratch) (void)hipFree(t->scratch);
    if (t->host_owned)
        for (char* sp : t->seg)
            if (sp) (void)hipHostFree(sp);
    delete t;
    return QOPS_OK;
}

int32_t qops_tier_segment_pointer(qops_tier* t, int32_t segment, void** host, size_t* bytes)
{
    if (!t || !host) return set_error(QOPS_INVALID_ARG, "null argument");
    if (segment < 0 || (size_t)segment >= t->seg.size()) return set_error(QOPS_INVALID_ARG, "segment out of range");
    *host = t->seg[(size_t)segment];
    if (bytes) *bytes = seg_bytes_of(t);
    return QOPS_OK;
}

int32_t qops_tier_init_basis(qops_tier* t, uint64_t x)
{
    if (!t) return set_error(QOPS_INVALID_ARG, "null handle");
    if (x >> t->n) return set_error(QOPS_INVALID_ARG, "basis index out of range");
    for (int q = 0; q < t->n; ++q) t->l2p[q] = q;
    t->basis = true;
    t->basis_x = x;
    return tier_copy_basis(t);
}

int32_t qops_tier_get_layout(qops_tier* t, int32_t* l2p)
{
    if (!t || !l2p) return set_error(QOPS_INVALID_ARG, "null argument");
    for (int q = 0; q < t->n; ++q) l2p[q] = t->l2p[q];
    return QOPS_OK;
}

int32_t qops_tier_plan(int32_t n, int32_t global_bits, int32_t max_active, const int32_t* l2p_in,
                       const qops_gate* gates, size_t n_gates, int32_t remap, qops_tier_stats* stats, int32_t* l2p_out)
{
    try {
        if (n < 2 || n > QOPS_MAX_QUBITS || global_bits < 1 || global_bits >= n || global_bits > 8 || max_active < 1 ||
            max_active > global_bits)
            return set_error(QOPS_INVALID_ARG, "bad tier shape");
        std::vector<int> l2p(n);
        for (int q = 0; q < n; ++q) l2p[q] = l2p_in ? l2p_in[q] : q;
        if (remap && !l2p_in) l2p = placement_from_counts(n, global_bits, gates, n_gates);
        PlanParams par;
        TierProgram prog;
        Err e = plan_tier(n, QOPS_C64, global_bits, max_active, l2p, gates, n_gates, remap != 0, par, false, prog);
        if (!e.ok()) return set_error(e.code, e.msg);
        fill_stats(prog, nullptr, stats);
        if (l2p_out)
            for (int q = 0; q < n; ++q) l2p_out[q] = prog.l2p_out[q];
        return QOPS_OK;
    } catch (...) {
        return set_error(QOPS_OUT_OF_MEMORY, "host allocation failed");
    }
}

int32_t qops_tier_run(qops_tier* t, const qops_gate* gates, size_t n_gates, const qops_tier_opts* opts,
                      qops_tier_stats* stats)
{
    try {
        if (!t) return set_error(QOPS_INVALID_ARG, "null handle");
        const int remap = opts ? opts->remap : 1;
        PlanParams par = params_from(opts ? &opts->plan : nullptr, t->nloc + t->amax, t->prec);
        if (opts && (opts->plan.mode == QOPS_PLAN_PROFILED || opts->plan.mode == QOPS_PLAN_LEARNED))
            par.mode = QOPS_PLAN_FUSED;   // group plans use the built-in widths
        if (remap && t->basis) {
            // a basis state may start in any layout: place it first (only
            // its one nonzero amplitude moves)
            put_one(t, basis_phys(t), false);
            t->l2p = placement_from_counts(t->n, t->g, gates, n_gates);
            put_one(t, basis_phys(t), true);
        }
        std::vector<int> l2p = t->l2p;
        TierProgram prog;
        Err e = plan_tier(t->n, t->prec, t->g, t->amax, l2p, gates, n_gates, remap != 0, par, true, prog);
        if (!e.ok()) return set_error(e.code, e.msg);
        // device images of every group plan before the pipeline starts (the
        // uploads are synchronous copies)
        for (TierStage& st : prog.stages)
            for (TierGroup& gr : st.groups) {
                int32_t urc = upload_plan(gr.plan);
                if (urc) {
                    for (TierStage& s2 : prog.stages)
                        for (TierGroup& g2 : s2.groups) free_plan_device(g2.plan);
                    return urc;
                }
            }
        const auto t0 = std::chrono::steady_clock::now();
        qops_sim sim;
        sim.prec = t->prec;
        sim.stream = t->stream;
        int32_t rc = QOPS_OK;
        size_t item = 0;
        for (size_t si = 0; si < prog.stages.size() && rc == QOPS_OK; ++si) {
            TierStage& st = prog.stages[si];
            for (size_t gi = 0; gi < st.groups.size() && rc == QOPS_OK; ++gi, ++item)
                rc = tier_group(t, st.groups[gi], (int)st.active.size(), item, gi == 0 && si > 0, sim);
        }
        hipError_t he = hipStreamSynchronize(t->copy_out);
        if (he == hipSuccess) he = hipStreamSynchronize(t->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(t->copy_in);
        sim.state = nullptr;   // borrowed slot, never freed by the handle
        for (TierStage& st : prog.stages)
            for (TierGroup& gr : st.groups) free_plan_device(gr.plan);
        if (rc) return rc;
        if (he != hipSuccess) return hip_fail(he, "tier run");
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        t->l2p = prog.l2p_out;
        t->basis = false;
        fill_stats(prog, t, stats);
        if (stats) stats->seconds = secs;
        return QOPS_OK;
    } catch (...) {
        return set_error(QOPS_OUT_OF_MEMORY, "host allocation failed");
    }
}

int32_t qops_tier_expect_z(qops_tier* t, double* out)
{
    try {
        if (!t || !out) return set_error(QOPS_INVALID_ARG, "null argument");
        const int nl = t->nloc;
        const size_t seg_bytes = ((size_t)1 << nl) * amp_size(t->prec);
        const size_t part = zsum_scratch_doubles(nl);
        const size_t need = 2 * (part + nl + 1);
        if (t->scratch_doubles < need) {
            if (t->scratch) (void)hipFree(t->scratch);
            t->scratch = nullptr;
            t->scratch_doubles = 0;
            hipError_t e = hipMalloc(&t->scratch, need * sizeof(double));
            if (e != hipSuccess) return hip_fail(e, "tier readout scratch");
            t->scratch_doubles = need;
        }
        const uint64_t nseg = 1ull << t->g;
        std::vector<double> sums((size_t)nseg * (nl + 1));
        hipError_t e = hipSuccess;
        for (uint64_t s = 0; s < nseg && e == hipSuccess; ++s) {
            const int slot = (int)(s & 1);
            if (s >= 2) e = hipStreamWaitEvent(t->copy_in, t->stored[slot], 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(t->dev[slot], t->seg[s], seg_bytes,
                                   hipMemcpyHostToDevice, t->copy_in);
            if (e == hipSuccess) e = hipEventRecord(t->loaded[slot], t->copy_in);
            if (e == hipSuccess) e = hipStreamWaitEvent(t->stream, t->loaded[slot], 0);
            double* sc = t->scratch + slot * (part + nl + 1);
            if (e == hipSuccess) e = launch_zsum(t->prec, t->dev[slot], nl, sc, sc + part, t->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(&sums[(size_t)s * (nl + 1)], sc + part, (nl + 1) * sizeof(double),
                                   hipMemcpyDeviceToHost, t->stream);
            if (e == hipSuccess) e = hipEventRecord(t->stored[slot], t->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
        if (e != hipSuccess) return hip_fail(e, "tier expect_z");
        // per physical bit: local bits from the segment sums, global bits from
        // the segments' totals (fixed order: segment by segment)
        std::vector<double> bit((size_t)t->n, 0.0);
        double total = 0.0;
        for (uint64_t s = 0; s < nseg; ++s) {
            const double* v = &sums[(size_t)s * (nl + 1)];
            total += v[0];
            for (int b = 0; b < nl; ++b) bit[b] += v[1 + b];
            for (int b = nl; b < t->n; ++b)
                if ((s >> (b - nl)) & 1ull) bit[b] += v[0];
        }
        for (int q = 0; q < t->n; ++q) out[q] = total - 2.0 * bit[t->l2p[q]];
        return QOPS_OK;
    } catch (...) {
        return set_error(QOPS_OUT_OF_MEMORY, "host allocation failed");
    }
}

int32_t qops_tier_read_state(qops_tier* t, void* host, int32_t order)
{
    if (!t || !host) return set_error(QOPS_INVALID_ARG, "null argument");
    hipError_t e = hipStreamSynchronize(t->copy_out);
    if (e != hipSuccess) return hip_fail(e, "tier read_state");
    const size_t asz = amp_size(t->prec);
    const size_t segb = seg_bytes_of(t);
    if (order == QOPS_ORDER_PHYSICAL) {
        for (size_t sgi = 0; sgi < t->seg.size(); ++sgi) std::memcpy(static_cast<char*>(host) + sgi * segb, t->seg[sgi], segb);
        return QOPS_OK;
    }
    if (order != QOPS_ORDER_LOGICAL) return set_error(QOPS_INVALID_ARG, "bad order");
    const uint64_t N = 1ull << t->n;
    char* dst = static_cast<char*>(host);
    for (uint64_t x = 0; x < N; ++x) {
        uint64_t p = 0;
        for (int q = 0; q < t->n; ++q)
            if ((x >> q) & 1ull) p |= 1ull << t->l2p[q];
        std::memcpy(dst + x * asz, amp_ptr(t, p), asz);
    }
    return QOPS_OK;
}

}  // extern "C"
