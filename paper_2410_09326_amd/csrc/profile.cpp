// Profiling run (paper Sec. III-C): counter-based and context-based records
// collected while the plan executes normally.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "profile.hpp"
#include "runtime.hpp"

using namespace qops;

namespace qops {

static void fill_record(const Plan& p, size_t i, qops_pass_record& r)
{
    const PassPlan& pp = p.passes[i];
    std::memset(&r, 0, sizeof(r));
    r.pass = (int32_t)i;
    r.type = (int32_t)pp.type;
    r.n_ops = (int32_t)pp.lop.size();
    int ng = 0;
    uint64_t mask = 0;
    for (int li : pp.lop) {
        ng += p.lops[li].nmerged;
        mask |= p.lops[li].tmask();
        if (p.lops[li].kind == LOp::DIAG)
            for (int j = 0; j < p.lops[li].k; ++j) mask |= 1ull << p.lops[li].t[j];
    }
    r.n_gates = ng;
    r.tile_bits = pp.L;
    r.n_mfma = pp.n_mfma;
    r.max_k = pp.max_k;
    r.n_remaps = pp.n_remaps;
    r.bytes_alg = pp.bytes_alg;
    r.flops = pp.flops;
    r.phys_mask = mask;
}

static void count_gates(const Plan& p, std::vector<int32_t>& lc, std::vector<int32_t>& pc)
{
    const int n = p.n;
    lc.assign((size_t)QOPS_NUM_KINDS * n, 0);
    pc.assign((size_t)QOPS_NUM_KINDS * n, 0);
    std::vector<int> l2p = p.l2p_in;
    for (const qops_gate& g : p.gates) {
        const int k = g.kind == QOPS_DENSE ? g.k : gate_arity(g.kind);
        for (int j = 0; j < k + g.n_ctrl; ++j) {
            const int q = j < k ? g.q[j] : g.ctrl[j - k];
            lc[(size_t)g.kind * n + q]++;
            pc[(size_t)g.kind * n + l2p[q]]++;
        }
        if (g.kind == QOPS_SWAP && g.n_ctrl == 0 && p.par.swap_mode == QOPS_SWAP_VIRTUAL) std::swap(l2p[g.q[0]], l2p[g.q[1]]);
    }
}

}  // namespace qops

extern "C" {

int32_t qops_profile_run(qops_sim* h, const qops_plan* plan, qops_profile** out)
{
    try {
        if (!h || !plan || !out) return set_error(QOPS_INVALID_ARG, "null argument");
        *out = nullptr;
        Plan& p = const_cast<qops_plan*>(plan)->p;
        int32_t rc = check_plan_matches(h, p);
        if (rc) return rc;
        rc = upload_plan(p);
        if (rc) return rc;
        const size_t np = p.passes.size();
        // events are created once per simulator and reused by later runs
        while (h->events.size() < np + 1) {
            hipEvent_t x;
            if (hipEventCreate(&x) != hipSuccess) return set_error(QOPS_HIP_ERROR, "event create");
            h->events.push_back(x);
        }
        const hipEvent_t* ev = h->events.data();
        hipError_t e = hipEventRecord(ev[0], h->stream);
        for (size_t i = 0; i < np && e == hipSuccess && rc == 0; ++i) {
            rc = launch_pass(h, p, p.passes[i]);
            if (rc == 0) e = hipEventRecord(ev[i + 1], h->stream);
        }
        if (e == hipSuccess && rc == 0) e = hipEventSynchronize(ev[np]);
        std::unique_ptr<qops_profile> pr(new qops_profile());
        pr->n = p.n;
        pr->prec = p.prec;
        pr->recs.resize(np);
        pr->feats.resize(np * kNumFeatures);
        for (size_t i = 0; i < np && e == hipSuccess && rc == 0; ++i) {
            fill_record(p, i, pr->recs[i]);
            float ms = 0, ms0 = 0;
            e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms0, ev[0], ev[i]);
            pr->recs[i].seconds = ms * 1e-3;
            pr->recs[i].t_begin = ms0 * 1e-3;
            pr->total += ms * 1e-3;
            pass_features(p, p.passes[i], &pr->feats[i * kNumFeatures]);
        }
        if (rc) return rc;
        if (e != hipSuccess) return hip_fail(e, "profiling run");
        count_gates(p, pr->lcount, pr->pcount);
        h->l2p = p.l2p_out;
        *out = pr.release();
        return QOPS_OK;
    } catch (...) {
        return set_error(QOPS_OUT_OF_MEMORY, "profiling run failed");
    }
}

int32_t qops_profile_num_passes(const qops_profile* pr, size_t* n)
{
    if (!pr || !n) return set_error(QOPS_INVALID_ARG, "null argument");
    *n = pr->recs.size();
    return QOPS_OK;
}

int32_t qops_profile_pass(const qops_profile* pr, size_t i, qops_pass_record* rec)
{
    if (!pr || !rec) return set_error(QOPS_INVALID_ARG, "null argument");
    if (i >= pr->recs.size()) return set_error(QOPS_INVALID_ARG, "pass index out of range");
    *rec = pr->recs[i];
    return QOPS_OK;
}

int32_t qops_profile_counts(const qops_profile* pr, int32_t* logical, int32_t* physical)
{
    if (!pr) return set_error(QOPS_INVALID_ARG, "null profile");
    if (logical) std::memcpy(logical, pr->lcount.data(), pr->lcount.size() * sizeof(int32_t));
    if (physical) std::memcpy(physical, pr->pcount.data(), pr->pcount.size() * sizeof(int32_t));
    return QOPS_OK;
}

int32_t qops_profile_total(const qops_profile* pr, double* seconds, int32_t* n)
{
    if (!pr) return set_error(QOPS_INVALID_ARG, "null profile");
    if (seconds) *seconds = pr->total;
    if (n) *n = pr->n;
    return QOPS_OK;
}

int32_t qops_profile_features(const qops_profile* pr, float* out)
{
    if (!pr || !out) return set_error(QOPS_INVALID_ARG, "null argument");
    std::memcpy(out, pr->feats.data(), pr->feats.size() * sizeof(float));
    return QOPS_OK;
}

int32_t qops_profile_dump(const qops_profile* pr, const char* path)
{
    if (!pr || !path) return set_error(QOPS_INVALID_ARG, "null argument");
    FILE* f = std::fopen(path, "w");
    if (!f) return set_error(QOPS_INVALID_ARG, std::string("cannot open ") + path);
    static const char* names[] = {"h", "x", "y", "z", "s", "sdg", "t", "tdg", "sx", "rx", "ry", "rz", "p", "u3",
                                  "cx", "cz", "cp", "swap", "rzz", "dense"};
    std::fprintf(f, "{\n  \"n\": %d,\n  \"precision\": \"%s\",\n  \"total_seconds\": %.9g,\n", pr->n,
                 pr->prec == QOPS_C64 ? "c64" : "c128", pr->total);
    std::fprintf(f, "  \"counters_logical\": {");
    bool first = true;
    const int n = pr->n;
    for (int k = 0; k < QOPS_NUM_KINDS && !pr->lcount.empty(); ++k) {
        bool any = false;
        for (int q = 0; q < n; ++q) any = any || pr->lcount[(size_t)k * n + q];
        if (!any) continue;
        std::fprintf(f, "%s\n    \"%s\": [", first ? "" : ",", names[k]);
        for (int q = 0; q < n; ++q) std::fprintf(f, "%s%d", q ? ", " : "", pr->lcount[(size_t)k * n + q]);
        std::fprintf(f, "]");
        first = false;
    }
    std::fprintf(f, "\n  },\n  \"passes\": [");
    for (size_t i = 0; i < pr->recs.size(); ++i) {
        const qops_pass_record& r = pr->recs[i];
        std::fprintf(f,
                     "%s\n    {\"pass\": %d, \"type\": %d, \"ops\": %d, \"gates\": %d, \"L\": %d, \"mfma\": %d, "
                     "\"max_k\": %d, \"remaps\": %d, \"t_begin\": %.9g, \"seconds\": %.9g, \"bytes\": %.6g, "
                     "\"flops\": %.6g, \"phys_mask\": %llu}",
                     i ? "," : "", r.pass, r.type, r.n_ops, r.n_gates, r.tile_bits, r.n_mfma, r.max_k, r.n_remaps,
                     r.t_begin, r.seconds, r.bytes_alg, r.flops, (unsigned long long)r.phys_mask);
    }
    std::fprintf(f, "\n  ]\n}\n");
    std::fclose(f);
    return QOPS_OK;
}

int32_t qops_profile_trace(const qops_profile* pr, const char* path)
{
    if (!pr || !path) return set_error(QOPS_INVALID_ARG, "null argument");
    FILE* f = std::fopen(path, "w");
    if (!f) return set_error(QOPS_INVALID_ARG, std::string("cannot open ") + path);
    static const char* kinds[] = {"register tile", "LDS tile", "whole state in LDS", "sweep", "bit swap"};
    const int nk = (int)(sizeof(kinds) / sizeof(kinds[0]));
    std::fprintf(f, "{\"displayTimeUnit\": \"ms\", \"traceEvents\": [\n");
    std::fprintf(f, "{\"name\": \"process_name\", \"ph\": \"M\", \"pid\": 1, \"args\": {\"name\": "
                    "\"qops %d qubits %s\"}},\n",
                 pr->n, pr->prec == QOPS_C64 ? "complex64" : "complex128");
    std::fprintf(f, "{\"name\": \"thread_name\", \"ph\": \"M\", \"pid\": 1, \"tid\": 1, \"args\": {\"name\": "
                    "\"passes\"}}");
    for (const qops_pass_record& r : pr->recs) {
        const char* kind = r.type >= 0 && r.type < nk ? kinds[r.type] : "pass";
        const double gbs = r.seconds > 0 ? r.bytes_alg / r.seconds / 1e9 : 0.0;
        std::fprintf(f,
                     ",\n{\"name\": \"%s\", \"cat\": \"pass\", \"ph\": \"X\", \"pid\": 1, \"tid\": 1, "
                     "\"ts\": %.3f, \"dur\": %.3f, \"args\": {\"pass\": %d, \"tile_bits\": %d, \"ops\": %d, "
                     "\"gates\": %d, \"mfma_ops\": %d, \"max_k\": %d, \"remaps\": %d, \"bytes\": %.6g, "
                     "\"flops\": %.6g, \"GB_per_s\": %.1f, \"phys_mask\": %llu}}",
                     kind, r.t_begin * 1e6, r.seconds * 1e6, r.pass, r.tile_bits, r.n_ops, r.n_gates, r.n_mfma,
                     r.max_k, r.n_remaps, r.bytes_alg, r.flops, gbs, (unsigned long long)r.phys_mask);
    }
    // gates per logical qubit (all kinds), as counters at t = 0
    const int n = pr->n;
    if (!pr->lcount.empty())
        for (int q = 0; q < n; ++q) {
            long long c = 0;
            for (int k = 0; k < QOPS_NUM_KINDS; ++k) c += pr->lcount[(size_t)k * n + q];
            std::fprintf(f, ",\n{\"name\": \"gates on q%d\", \"ph\": \"C\", \"pid\": 1, \"ts\": 0, "
                            "\"args\": {\"gates\": %lld}}",
                         q, c);
        }
    std::fprintf(f, "\n]}\n");
    const bool ok = std::ferror(f) == 0;
    std::fclose(f);
    if (!ok) return set_error(QOPS_INVALID_ARG, std::string("write failed: ") + path);
    return QOPS_OK;
}

int32_t qops_profile_merge(qops_profile* dst, const qops_profile* src)
{
    if (!dst || !src) return set_error(QOPS_INVALID_ARG, "null argument");
    dst->recs.insert(dst->recs.end(), src->recs.begin(), src->recs.end());
    dst->feats.insert(dst->feats.end(), src->feats.begin(), src->feats.end());
    dst->total += src->total;
    if (dst->lcount.size() == src->lcount.size()) {
        for (size_t i = 0; i < dst->lcount.size(); ++i) {
            dst->lcount[i] += src->lcount[i];
            dst->pcount[i] += src->pcount[i];
        }
    }
    return QOPS_OK;
}

int32_t qops_profile_create(int32_t n, qops_profile** out)
{
    if (!out || n < 1 || n > QOPS_MAX_QUBITS) return set_error(QOPS_INVALID_ARG, "bad arguments");
    qops_profile* p = new qops_profile();
    p->n = n;
    p->lcount.assign((size_t)QOPS_NUM_KINDS * n, 0);
    p->pcount.assign((size_t)QOPS_NUM_KINDS * n, 0);
    *out = p;
    return QOPS_OK;
}

int32_t qops_profile_save(const qops_profile* pr, const char* path)
{
    if (!pr || !path) return set_error(QOPS_INVALID_ARG, "null argument");
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(QOPS_INVALID_ARG, std::string("cannot open ") + path);
    const char magic[8] = {'Q', 'O', 'P', 'S', 'P', 'R', 'F', '1'};
    const uint64_t nr = pr->recs.size(), nc = pr->lcount.size();
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&pr->n, 4, 1, f) == 1 && std::fwrite(&pr->prec, 4, 1, f) == 1 &&
              std::fwrite(&pr->total, 8, 1, f) == 1 && std::fwrite(&nr, 8, 1, f) == 1 && std::fwrite(&nc, 8, 1, f) == 1 &&
              std::fwrite(pr->recs.data(), sizeof(qops_pass_record), nr, f) == nr &&
              std::fwrite(pr->feats.data(), sizeof(float), nr * kNumFeatures, f) == nr * kNumFeatures &&
              std::fwrite(pr->lcount.data(), 4, nc, f) == nc && std::fwrite(pr->pcount.data(), 4, nc, f) == nc;
    std::fclose(f);
    return ok ? QOPS_OK : set_error(QOPS_INVALID_ARG, "write failed");
}

int32_t qops_profile_load(const char* path, qops_profile** out)
{
    if (!path || !out) return set_error(QOPS_INVALID_ARG, "null argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(QOPS_INVALID_ARG, std::string("cannot open ") + path);
    std::unique_ptr<qops_profile> p(new qops_profile());
    char magic[8];
    uint64_t nr = 0, nc = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "QOPSPRF1", 8) == 0 &&
              std::fread(&p->n, 4, 1, f) == 1 && std::fread(&p->prec, 4, 1, f) == 1 && std::fread(&p->total, 8, 1, f) == 1 &&
              std::fread(&nr, 8, 1, f) == 1 && std::fread(&nc, 8, 1, f) == 1 && nr < (1ull << 28) && nc < (1ull << 20);
    if (ok) {
        p->recs.resize(nr);
        p->feats.resize(nr * kNumFeatures);
        p->lcount.resize(nc);
        p->pcount.resize(nc);
        ok = std::fread(p->recs.data(), sizeof(qops_pass_record), nr, f) == nr &&
             std::fread(p->feats.data(), sizeof(float), nr * kNumFeatures, f) == nr * kNumFeatures &&
             std::fread(p->lcount.data(), 4, nc, f) == nc && std::fread(p->pcount.data(), 4, nc, f) == nc;
    }
    std::fclose(f);
    if (!ok) return set_error(QOPS_INVALID_ARG, "not a qops profile file");
    *out = p.release();
    return QOPS_OK;
}

int32_t qops_profile_free(qops_profile* pr)
{
    delete pr;
    return QOPS_OK;
}

}  // extern "C"
