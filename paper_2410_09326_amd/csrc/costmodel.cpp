// Plan pricing: candidate plans (tile widths x qubit remap) are priced by a
// cost model and the cheapest is kept -- the profile-guided activation of an
// optimisation (paper Sec. III-D), with the profile's measured pass times as
// the plain cost table and a trained perceptron as the learned one.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "mlp.hpp"
#include "profile.hpp"
#include "runtime.hpp"

namespace qops {

// Plain cost table (the profile-guided table of measured costs): a pass's
// time per amplitude, looked up by the shape of the pass -- its kernel kind,
// tile width, register/wave split, widest dense block and number of device
// operations (exact up to 16, then powers of two) -- as the median over the
// profile's passes of that shape.  Shapes the profile never saw fall back to
// coarser keys (dropping the wave split, then bucketing the operation count
// by powers of two, then the block width) and finally to the median of the
// pass kind.  On a GPU every pass streams the whole state, so the high bits
// a pass touches (the paper's stride) matter little; what it carries does.
namespace {

int feat_round(float v, float scale) { return (int)std::lround((double)v * scale); }

struct PassShape {
    int type, L, W, maxk, nops;
};

PassShape shape_of(const float* f)
{
    PassShape s;
    s.type = 0;
    for (int t = 0; t < 5; ++t)
        if (f[2 + t] > 0.5f) s.type = t;
    s.L = feat_round(f[7], 16.f);
    s.W = feat_round(f[16], 1.f);
    s.maxk = feat_round(f[14], 6.f);
    s.nops = feat_round(f[54], 64.f);
    return s;
}

int ops_bucket(int nops, bool fine)
{
    if (fine && nops <= 16) return nops;
    int b = 17;
    for (int v = 32; v <= nops; v <<= 1) ++b;
    return fine ? b : (nops <= 1 ? 0 : 1 + (31 - __builtin_clz((unsigned)nops)));
}

// key levels, finest first
uint64_t shape_key(const PassShape& s, int level)
{
    uint64_t k = (uint64_t)s.type;
    if (level <= 3) k = k * 64 + (uint64_t)s.L;
    if (level <= 0) k = k * 8 + (uint64_t)s.W;
    if (level <= 2) k = k * 8 + (uint64_t)s.maxk;
    if (level <= 1) k = k * 64 + (uint64_t)ops_bucket(s.nops, level == 0);
    return k * 8 + (uint64_t)level;
}
constexpr int kLevels = 5;

double amp_scale(const float* f)
{
    const double n = std::round((double)f[0] * 32.0);
    return std::ldexp(1.0, (int)n - 30);
}

double median(std::vector<double>& v)
{
    const size_t m = v.size() / 2;
    std::nth_element(v.begin(), v.begin() + (long)m, v.end());
    double x = v[m];
    if (v.size() % 2 == 0) {
        const double lo = *std::max_element(v.begin(), v.begin() + (long)m);
        x = 0.5 * (x + lo);
    }
    return x;
}

}  // namespace

struct PlainTable {
    std::unordered_map<uint64_t, double> cost;   // seconds at 30 qubits
};

static bool fit_plain(const qops_profile& pr, PlainTable& tab)
{
    const size_t np = pr.recs.size();
    if (np == 0) return false;
    std::unordered_map<uint64_t, std::vector<double>> bins;
    for (size_t i = 0; i < np; ++i) {
        const float* f = &pr.feats[i * kNumFeatures];
        const PassShape s = shape_of(f);
        const double y = pr.recs[i].seconds / amp_scale(f);
        for (int lv = 0; lv < kLevels; ++lv) bins[shape_key(s, lv)].push_back(y);
    }
    tab.cost.clear();
    for (auto& kv : bins) tab.cost[kv.first] = median(kv.second);
    return true;
}

static double plain_predict(const PlainTable& tab, const float* f)
{
    const PassShape s = shape_of(f);
    for (int lv = 0; lv < kLevels; ++lv) {
        auto it = tab.cost.find(shape_key(s, lv));
        if (it != tab.cost.end()) return it->second * amp_scale(f);
    }
    return 2e-6;   // no pass of this kind profiled: a launch's floor
}

// The network predicts ln(seconds) scaled to 30 qubits; f[0] is n / 32.
static double learned_seconds(float y, const float* f)
{
    const double n = std::round((double)f[0] * 32.0);
    return std::exp((double)y + (n - 30.0) * 0.69314718055994530942);
}

static double price(const Plan& p, const qops_plan_opts* o, const PlainTable& theta)
{
    std::vector<float> f(p.passes.size() * kNumFeatures);
    for (size_t i = 0; i < p.passes.size(); ++i) pass_features(p, p.passes[i], &f[i * kNumFeatures]);
    double t = 0;
    if (o->mode == QOPS_PLAN_LEARNED && o->model) {
        std::vector<float> y(p.passes.size());
        mlp_predict_host(o->model, f.data(), (int)p.passes.size(), y.data());
        for (size_t i = 0; i < p.passes.size(); ++i) t += learned_seconds(y[i], &f[i * kNumFeatures]);
    } else {
        for (size_t i = 0; i < p.passes.size(); ++i) t += plain_predict(theta, &f[i * kNumFeatures]);
    }
    return t;
}

int32_t build_priced_plan(int n, int prec, const int32_t* l2p, const qops_gate* g, size_t ng,
                          const qops_plan_opts* opts, Plan& out)
{
    PlanParams par = params_from(opts, n, prec);
    const bool priced = opts && (opts->mode == QOPS_PLAN_PROFILED || opts->mode == QOPS_PLAN_LEARNED);
    if (!priced) {
        Err e = build_plan(n, prec, l2p, g, ng, par, out);
        if (!e.ok()) return set_error(e.code, e.msg);
        return QOPS_OK;
    }
    const bool learned = opts->mode == QOPS_PLAN_LEARNED && opts->model;
    PlainTable theta;
    if (!learned) {
        if (!opts->profile) return set_error(QOPS_INVALID_ARG, "PROFILED mode needs a profile (opts.profile)");
        if (!fit_plain(*opts->profile, theta)) return set_error(QOPS_INVALID_ARG, "profile has no usable pass records");
    }
    const auto t0 = std::chrono::steady_clock::now();
    double best = -1;
    // candidates: tile width above the six lane bits (0 = the default
    // widths: small register tiles, the largest LDS tile) x qubit remap x
    // block fusion width (a fixed fusion width in the options is kept)
    const int max_up = prec == QOPS_C64 ? 7 : 6;
    const int k_lo = opts->max_fuse_k > 0 ? opts->max_fuse_k : 1;
    const int k_hi = opts->max_fuse_k > 0 ? opts->max_fuse_k : 4;
    std::vector<int> widths;
    if (prec == QOPS_C64) widths.push_back(0);   // for complex128 the default equals width 6
    for (int up = 4; up <= max_up; ++up) widths.push_back(up);
    for (int kf = k_lo; kf <= k_hi; ++kf)
        for (int remap = 0; remap <= 1; ++remap)
            for (int up : widths) {
                qops_plan_opts o = *opts;
                o.tile_upper = up;
                o.max_fuse_k = kf;
                PlanParams cp = params_from(&o, n, prec);
                cp.mode = QOPS_PLAN_FUSED;
                cp.remap = remap;
                Plan cand;
                Err e = build_plan(n, prec, l2p, g, ng, cp, cand);
                if (!e.ok()) return set_error(e.code, e.msg);
                const double t = price(cand, opts, theta);
                if (best < 0 || t < best) {
                    best = t;
                    out = std::move(cand);
                    out.predicted_s = t;
                }
            }
    out.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return QOPS_OK;
}

}  // namespace qops

extern "C" {

int32_t qops_plan_predict(const qops_plan* p, const qops_plan_opts* opts, double* seconds)
{
    if (!p || !opts || !seconds) return qops::set_error(QOPS_INVALID_ARG, "null argument");
    qops::PlainTable theta;
    if (!(opts->mode == QOPS_PLAN_LEARNED && opts->model)) {
        if (!opts->profile || !qops::fit_plain(*opts->profile, theta))
            return qops::set_error(QOPS_INVALID_ARG, "need a model (LEARNED) or a profile");
    }
    *seconds = qops::price(p->p, opts, theta);
    return QOPS_OK;
}

int32_t qops_profile_compact(const qops_profile* src, qops_profile** out)
{
    try {
        if (!src || !out) return qops::set_error(QOPS_INVALID_ARG, "null argument");
        *out = nullptr;
        // per finest shape: the passes at the 10th, 30th, 50th, 70th and 90th
        // percentile of the per-amplitude time (all of them if fewer than 5)
        std::unordered_map<uint64_t, std::vector<std::pair<double, size_t>>> bins;
        for (size_t i = 0; i < src->recs.size(); ++i) {
            const float* f = &src->feats[i * qops::kNumFeatures];
            bins[qops::shape_key(qops::shape_of(f), 0)].push_back({src->recs[i].seconds / qops::amp_scale(f), i});
        }
        std::vector<uint64_t> keys;
        for (auto& kv : bins) keys.push_back(kv.first);
        std::sort(keys.begin(), keys.end());
        std::unique_ptr<qops_profile> c(new qops_profile());
        c->n = src->n;
        c->prec = src->prec;
        c->lcount = src->lcount;
        c->pcount = src->pcount;
        for (uint64_t k : keys) {
            auto& v = bins[k];
            std::sort(v.begin(), v.end());
            std::vector<size_t> pick;
            if (v.size() <= 5) {
                for (auto& e : v) pick.push_back(e.second);
            } else {
                for (double qn : {0.1, 0.3, 0.5, 0.7, 0.9}) pick.push_back(v[(size_t)(qn * (double)(v.size() - 1) + 0.5)].second);
            }
            for (size_t i : pick) {
                c->recs.push_back(src->recs[i]);
                c->feats.insert(c->feats.end(), src->feats.begin() + (long)(i * qops::kNumFeatures),
                                src->feats.begin() + (long)((i + 1) * qops::kNumFeatures));
                c->total += src->recs[i].seconds;
            }
        }
        *out = c.release();
        return QOPS_OK;
    } catch (...) {
        return qops::set_error(QOPS_OUT_OF_MEMORY, "host allocation failed");
    }
}

int32_t qops_profile_predict_passes(const qops_profile* pr, const qops_plan_opts* opts, double* out)
{
    if (!pr || !opts || !out) return qops::set_error(QOPS_INVALID_ARG, "null argument");
    const size_t np = pr->recs.size();
    if (opts->mode == QOPS_PLAN_LEARNED && opts->model) {
        std::vector<float> y(np);
        qops::mlp_predict_host(opts->model, pr->feats.data(), (int)np, y.data());
        for (size_t i = 0; i < np; ++i) out[i] = qops::learned_seconds(y[i], &pr->feats[i * qops::kNumFeatures]);
        return QOPS_OK;
    }
    qops::PlainTable theta;
    if (!opts->profile || !qops::fit_plain(*opts->profile, theta))
        return qops::set_error(QOPS_INVALID_ARG, "need a model (LEARNED) or a profile");
    for (size_t i = 0; i < np; ++i) out[i] = qops::plain_predict(theta, &pr->feats[i * qops::kNumFeatures]);
    return QOPS_OK;
}

}  // extern "C"
