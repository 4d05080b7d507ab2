// Circuit IR, layout tracking and the fusion planner (host side).
#pragma once
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qops.h"
#include "devprog.hpp"

namespace qops {

using cd = std::complex<double>;

// A gate lowered onto PHYSICAL bits.
struct LOp {
    enum Kind { ONEQ = 0, DIAG = 1, DENSE = 2, PSWAP = 3 } kind = ONEQ;
    int k = 0;                 // ONEQ 1; DENSE k; DIAG number of table bits; PSWAP 2
    int t[10] = {0};           // ONEQ/DENSE targets (matrix bit order); DIAG table bits; PSWAP the two bits
    uint64_t cmask = 0;        // ONEQ/DENSE controls (physical mask)
    std::vector<cd> m;         // 2x2 / 2^k x 2^k row-major / 2^k diagonal table
    int gate = -1;             // first source gate
    int gkind = -1;            // kind of the first source gate
    int nmerged = 1;           // source gates folded into this op
    bool cphase = false;       // DIAG: table is 1 except its last entry (all bits 1)
    bool dead = false;
    uint64_t touch() const;    // every physical bit the op reads or conditions on
    uint64_t tmask() const;    // non-diagonal target bits (ONEQ/DENSE/PSWAP)
};

enum PassType { PASS_TILE_REG = 0, PASS_TILE_LDS = 1, PASS_STATE_LDS = 2, PASS_SWEEP = 3, PASS_SWAP_BITS = 4 };

struct PassPlan {
    PassType type = PASS_TILE_REG;
    int R = 0, W = 0, L = 0;
    std::vector<int> up;       // upper tile bits (physical)
    std::vector<int> lop;      // indices into Plan::lops
    int hdr = -1;              // index into Plan::hdrs (tile passes)
    int op0 = 0, nops = 0;     // range in Plan::dops
    int swap_a = 0, swap_b = 0;
    double bytes_alg = 0;      // algorithmic HBM bytes
    double flops = 0;
    int n_lane_ops = 0, n_reg_ops = 0, n_diag_ops = 0, n_remaps = 0, n_dense = 0, n_mfma = 0, max_k = 0;
};

struct PlanParams {
    int mode = QOPS_PLAN_FUSED;
    int swap_mode = QOPS_SWAP_VIRTUAL;
    int R = 5, W = 2;          // register-tile variant
    int L_lds = 13;            // LDS-tile bits
    int max_fuse_k = 1;
    int use_mfma = 1;
    int state_lds_max_n = 12;  // whole state in one work-group's LDS up to this n
    int check_unitary = 0;
    int remap = 0;             // move the most-targeted qubits into physical bits 0..5 first
    int force_lds = 0;         // every tile pass is an LDS pass (batched executor)
    int fold = 0;              // rotation folding: 1 on, -1 off, 0 by the T-gate rule
    int merge_blocks = 0;      // priced dense-block merging: -1 off, else on
};

struct Plan {
    int n = 0, prec = 0;
    PlanParams par;
    std::vector<int> l2p_in, l2p_out;
    std::vector<qops_gate> gates;      // copy of the input (mat pointers into mats)
    std::vector<std::vector<double>> mats;
    std::vector<LOp> lops;
    std::vector<PassPlan> passes;
    std::vector<PassHdr> hdrs;
    std::vector<DevOp> dops;
    std::vector<double> coef;          // FP64 image; cast to the state precision at upload
    int n_virtual_swaps = 0;
    int n_folded = 0;                  // phase gates removed by rotation folding
    double plan_seconds = 0;
    double predicted_s = 0;
    // device copies (uploaded lazily by the runtime)
    void* d_hdr = nullptr;
    void* d_ops = nullptr;
    void* d_coef = nullptr;
    bool dirty = true;
};

// Status with message (thread-local last error is set by the ABI layer).
struct Err {
    int code = 0;
    std::string msg;
    bool ok() const { return code == 0; }
};

int gate_arity(int kind);
bool diag_kind(int kind);
// Rotation folding over phase polynomials; `removed` = input phase gates
// minus the phase gates of the result.
bool fold_rule_fires(const qops_gate* g, size_t ng);
void fold_rotations(int n, const qops_gate* in, size_t ng, std::vector<qops_gate>& out, int& removed);
// The gate's matrix (ordered targets, little-endian bit order), FP64.
Err gate_matrix(const qops_gate& g, std::vector<cd>& out);
Err validate_gates(int n, const qops_gate* g, size_t ng, bool check_unitary);

// Builds a plan (validation, lowering with the running layout, merging,
// packing, device program emission).
Err build_plan(int n, int prec, const int32_t* l2p_in, const qops_gate* g, size_t ng, const PlanParams& par,
               Plan& out);
// Lowers gates onto physical bits with the running layout l2p (updated in
// place; unconditioned SWAPs are layout updates in VIRTUAL mode).
Err lower_gates(int n, const qops_gate* g, size_t ng, int swap_mode, std::vector<int>& l2p, std::vector<LOp>& out,
                int& nvirt);
// Plans already-lowered operations on an n-bit state in identity layout
// (merging, fusion, packing, device program); `ops` is consumed.
Err plan_from_lops(int n, int prec, std::vector<LOp>& ops, const PlanParams& par, Plan& p);
// Rebinds angles/matrices (same structure) and re-emits coefficients.
Err update_plan(Plan& p, const qops_gate* g, size_t ng);

// Per-pass features for the cost models (64 floats per pass).
void pass_features(const Plan& p, const PassPlan& pp, float* f64);
constexpr int kNumFeatures = 64;

}  // namespace qops
