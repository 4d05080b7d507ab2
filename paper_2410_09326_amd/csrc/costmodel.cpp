// Plan pricing: candidate plans (tile widths x qubit remap) are priced by a
// cost model and the cheapest is kept -- the profile-guided activation of an
// optimisation (paper Sec. III-D), with the profile's measured pass times as
// the plain cost table and a trained perceptron as the learned one.
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mlp.hpp"
#include "profile.hpp"
#include "runtime.hpp"

namespace qops {

// Plain cost table: pass time / (2^n / 2^30) fitted as a linear function of
// a few pass features (pass type, operation counts by class, matrix-core
// flops, tile shape) by least squares over the profile's pass records.
static const int kPlainIdx[] = {2, 3, 4, 5, 6, 8, 9, 10, 11, 12, 13, 15, 16, 17, 62};
static constexpr int kPlainDim = sizeof(kPlainIdx) / sizeof(int);

static bool solve_spd(std::vector<double>& A, std::vector<double>& b, int d)
{
    // Cholesky with a small ridge for rank-deficient designs
    for (int i = 0; i < d; ++i) A[i * d + i] += 1e-9 + 1e-6 * A[i * d + i];
    for (int j = 0; j < d; ++j) {
        double s = A[j * d + j];
        for (int k = 0; k < j; ++k) s -= A[j * d + k] * A[j * d + k];
        if (s <= 0) return false;
        A[j * d + j] = std::sqrt(s);
        for (int i = j + 1; i < d; ++i) {
            double t = A[i * d + j];
            for (int k = 0; k < j; ++k) t -= A[i * d + k] * A[j * d + k];
            A[i * d + j] = t / A[j * d + j];
        }
    }
    for (int i = 0; i < d; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= A[i * d + k] * b[k];
        b[i] = t / A[i * d + i];
    }
    for (int i = d - 1; i >= 0; --i) {
        double t = b[i];
        for (int k = i + 1; k < d; ++k) t -= A[k * d + i] * b[k];
        b[i] = t / A[i * d + i];
    }
    return true;
}

static bool fit_plain(const qops_profile& pr, std::vector<double>& theta)
{
    const size_t np = pr.recs.size();
    if (np == 0) return false;
    const int d = kPlainDim;
    std::vector<double> A((size_t)d * d, 0.0), b(d, 0.0);
    for (size_t i = 0; i < np; ++i) {
        const float* f = &pr.feats[i * kNumFeatures];
        const double n = f[0] * 32.0;
        const double scale = std::ldexp(1.0, (int)std::lround(n) - 30);
        const double y = pr.recs[i].seconds / scale;
        double x[kPlainDim];
        for (int j = 0; j < d; ++j) x[j] = f[kPlainIdx[j]];
        for (int r = 0; r < d; ++r) {
            b[r] += x[r] * y;
            for (int c = 0; c < d; ++c) A[(size_t)r * d + c] += x[r] * x[c];
        }
    }
    if (!solve_spd(A, b, d)) return false;
    theta = b;
    return true;
}

double plain_predict(const std::vector<double>& theta, const float* f)
{
    const double n = f[0] * 32.0;
    const double scale = std::ldexp(1.0, (int)std::lround(n) - 30);
    double y = 0;
    for (int j = 0; j < kPlainDim; ++j) y += theta[j] * f[kPlainIdx[j]];
    const double floor_s = 2e-6;   // a launch never costs less than this
    return std::max(y * scale, floor_s);
}

// The network predicts ln(seconds) scaled to 30 qubits; f[0] is n / 32.
static double learned_seconds(float y, const float* f)
{
    const double n = std::round((double)f[0] * 32.0);
    return std::exp((double)y + (n - 30.0) * 0.69314718055994530942);
}

static double price(const Plan& p, const qops_plan_opts* o, const std::vector<double>& theta)
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
    std::vector<double> theta;
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
    std::vector<double> theta;
    if (!(opts->mode == QOPS_PLAN_LEARNED && opts->model)) {
        if (!opts->profile || !qops::fit_plain(*opts->profile, theta))
            return qops::set_error(QOPS_INVALID_ARG, "need a model (LEARNED) or a profile");
    }
    *seconds = qops::price(p->p, opts, theta);
    return QOPS_OK;
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
    std::vector<double> theta;
    if (!opts->profile || !qops::fit_plain(*opts->profile, theta))
        return qops::set_error(QOPS_INVALID_ARG, "need a model (LEARNED) or a profile");
    for (size_t i = 0; i < np; ++i) out[i] = qops::plain_predict(theta, &pr->feats[i * qops::kNumFeatures]);
    return QOPS_OK;
}

}  // extern "C"
