// Circuit IR validation, virtual-swap layout tracking, gate merging and tile
// packing.  Produces the device programs the kernels execute.
//
// Paper correspondence:
//   * virtual swap (Sec. III-D): a SWAP exchanges two entries of the
//     logical-to-physical map and moves no amplitude;
//   * single-qubit gate merging (Sec. III-D): a run of one-qubit gates on a
//     qubit becomes one 2x2 unitary (composed in FP64);
//   * chunk-segment-aware updating (Sec. II-B): gates whose targets fall in
//     the buffered segment are cheap, so consecutive gates are packed into
//     one pass over a tile whose qubit set covers all of their targets.
#include "planner.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace qops {

uint64_t LOp::touch() const
{
    uint64_t m = cmask;
    for (int j = 0; j < k; ++j) m |= 1ull << t[j];
    return m;
}

uint64_t LOp::tmask() const
{
    if (kind == DIAG) return 0;
    uint64_t m = 0;
    for (int j = 0; j < k; ++j) m |= 1ull << t[j];
    return m;
}

int gate_arity(int kind)
{
    if (kind >= QOPS_H && kind <= QOPS_U3) return 1;
    if (kind >= QOPS_CX && kind <= QOPS_RZZ) return 2;
    if (kind == QOPS_DENSE) return 0;
    return -1;
}

bool diag_kind(int kind)
{
    switch (kind) {
    case QOPS_Z: case QOPS_S: case QOPS_SDG: case QOPS_T: case QOPS_TDG: case QOPS_RZ: case QOPS_P:
    case QOPS_CZ: case QOPS_CP: case QOPS_RZZ:
        return true;
    default:
        return false;
    }
}

static Err mkerr(int code, const std::string& m)
{
    Err e;
    e.code = code;
    e.msg = m;
    return e;
}

Err gate_matrix(const qops_gate& g, std::vector<cd>& m)
{
    const double r2 = 1.0 / std::sqrt(2.0);
    const cd I(0, 1);
    const int k = g.kind == QOPS_DENSE ? g.k : gate_arity(g.kind);
    if (k < 1 || k > QOPS_MAX_K) return mkerr(QOPS_UNSUPPORTED, "gate arity out of range");
    const int d = 1 << k;
    m.assign((size_t)d * d, cd(0, 0));
    auto at = [&](int r, int c) -> cd& { return m[(size_t)r * d + c]; };
    const double th = g.param[0];
    const double c = std::cos(th / 2), s = std::sin(th / 2);
    switch (g.kind) {
    case QOPS_H: at(0, 0) = r2; at(0, 1) = r2; at(1, 0) = r2; at(1, 1) = -r2; break;
    case QOPS_X: at(0, 1) = 1; at(1, 0) = 1; break;
    case QOPS_Y: at(0, 1) = -I; at(1, 0) = I; break;
    case QOPS_Z: at(0, 0) = 1; at(1, 1) = -1; break;
    case QOPS_S: at(0, 0) = 1; at(1, 1) = I; break;
    case QOPS_SDG: at(0, 0) = 1; at(1, 1) = -I; break;
    case QOPS_T: at(0, 0) = 1; at(1, 1) = std::polar(1.0, M_PI / 4); break;
    case QOPS_TDG: at(0, 0) = 1; at(1, 1) = std::polar(1.0, -M_PI / 4); break;
    case QOPS_SX: at(0, 0) = cd(0.5, 0.5); at(0, 1) = cd(0.5, -0.5); at(1, 0) = cd(0.5, -0.5); at(1, 1) = cd(0.5, 0.5); break;
    case QOPS_RX: at(0, 0) = c; at(0, 1) = -I * s; at(1, 0) = -I * s; at(1, 1) = c; break;
    case QOPS_RY: at(0, 0) = c; at(0, 1) = -s; at(1, 0) = s; at(1, 1) = c; break;
    case QOPS_RZ: at(0, 0) = std::polar(1.0, -th / 2); at(1, 1) = std::polar(1.0, th / 2); break;
    case QOPS_P: at(0, 0) = 1; at(1, 1) = std::polar(1.0, th); break;
    case QOPS_U3: {
        const double ph = g.param[1], la = g.param[2];
        at(0, 0) = c;
        at(0, 1) = -std::polar(s, la);
        at(1, 0) = std::polar(s, ph);
        at(1, 1) = std::polar(c, ph + la);
        break;
    }
    case QOPS_CX: at(0, 0) = 1; at(2, 2) = 1; at(1, 3) = 1; at(3, 1) = 1; break;
    case QOPS_CZ: at(0, 0) = 1; at(1, 1) = 1; at(2, 2) = 1; at(3, 3) = -1; break;
    case QOPS_CP: at(0, 0) = 1; at(1, 1) = 1; at(2, 2) = 1; at(3, 3) = std::polar(1.0, th); break;
    case QOPS_SWAP: at(0, 0) = 1; at(1, 2) = 1; at(2, 1) = 1; at(3, 3) = 1; break;
    case QOPS_RZZ:
        at(0, 0) = std::polar(1.0, -th / 2); at(1, 1) = std::polar(1.0, th / 2);
        at(2, 2) = std::polar(1.0, th / 2); at(3, 3) = std::polar(1.0, -th / 2); break;
    case QOPS_DENSE:
        if (!g.mat) return mkerr(QOPS_INVALID_ARG, "DENSE gate without a matrix");
        for (int i = 0; i < d * d; ++i) m[i] = cd(g.mat[2 * i], g.mat[2 * i + 1]);
        break;
    default:
        return mkerr(QOPS_INVALID_ARG, "unknown gate kind");
    }
    return Err{};
}

Err validate_gates(int n, const qops_gate* g, size_t ng, bool check_unitary)
{
    if (ng > 0 && !g) return mkerr(QOPS_INVALID_ARG, "null gate list");
    for (size_t i = 0; i < ng; ++i) {
        const qops_gate& x = g[i];
        const std::string at = " (gate " + std::to_string(i) + ")";
        if (x.kind >= QOPS_NUM_KINDS) return mkerr(QOPS_INVALID_ARG, "unknown gate kind" + at);
        const int ar = gate_arity(x.kind);
        const int k = x.kind == QOPS_DENSE ? x.k : ar;
        if (x.kind == QOPS_DENSE) {
            if (x.k < 1 || x.k > QOPS_MAX_K) return mkerr(QOPS_UNSUPPORTED, "DENSE k must be 1..6" + at);
            if (!x.mat) return mkerr(QOPS_INVALID_ARG, "DENSE gate without a matrix" + at);
        } else if (x.k != ar) {
            return mkerr(QOPS_INVALID_ARG, "k does not match the gate kind" + at);
        }
        if (x.n_ctrl > QOPS_MAX_CTRL) return mkerr(QOPS_UNSUPPORTED, "more than 4 controls" + at);
        if (diag_kind(x.kind) && k + x.n_ctrl > 6)
            return mkerr(QOPS_UNSUPPORTED, "diagonal gate with more than 6 qubits" + at);
        uint64_t seen = 0;
        for (int j = 0; j < k + x.n_ctrl; ++j) {
            const int q = j < k ? x.q[j] : x.ctrl[j - k];
            if (q < 0 || q >= n) return mkerr(QOPS_QUBIT_RANGE, "qubit out of range" + at);
            if (seen & (1ull << q)) return mkerr(QOPS_DUPLICATE_QUBIT, "qubit listed twice" + at);
            seen |= 1ull << q;
        }
        if (check_unitary && x.kind == QOPS_DENSE) {
            std::vector<cd> m;
            Err e = gate_matrix(x, m);
            if (!e.ok()) return e;
            const int d = 1 << k;
            double worst = 0;
            for (int r = 0; r < d; ++r)
                for (int c2 = 0; c2 < d; ++c2) {
                    cd acc = 0;
                    for (int s = 0; s < d; ++s) acc += std::conj(m[(size_t)s * d + r]) * m[(size_t)s * d + c2];
                    worst = std::max(worst, std::abs(acc - (r == c2 ? cd(1) : cd(0))));
                }
            if (worst > 1e-9) return mkerr(QOPS_NOT_UNITARY, "DENSE matrix is not unitary" + at);
        }
    }
    return Err{};
}

// ---------------------------------------------------------------------------
// Lowering: logical gates -> physical ops, with the running layout
// ---------------------------------------------------------------------------

static Err lower(int n, const qops_gate* g, size_t ng, int swap_mode, std::vector<int>& l2p, std::vector<LOp>& out,
                 int& nvirt)
{
    (void)n;
    std::vector<cd> u;
    for (size_t i = 0; i < ng; ++i) {
        const qops_gate& x = g[i];
        const int k = x.kind == QOPS_DENSE ? x.k : gate_arity(x.kind);
        int pt[6];
        for (int j = 0; j < k; ++j) pt[j] = l2p[x.q[j]];
        uint64_t cm = 0;
        for (int j = 0; j < x.n_ctrl; ++j) cm |= 1ull << l2p[x.ctrl[j]];
        if (x.kind == QOPS_SWAP && x.n_ctrl == 0) {
            if (swap_mode == QOPS_SWAP_VIRTUAL) {
                std::swap(l2p[x.q[0]], l2p[x.q[1]]);
                ++nvirt;
            } else {
                LOp o;
                o.kind = LOp::PSWAP;
                o.k = 2;
                o.t[0] = pt[0];
                o.t[1] = pt[1];
                o.gate = (int)i;
                o.gkind = x.kind;
                out.push_back(o);
            }
            continue;
        }
        Err e = gate_matrix(x, u);
        if (!e.ok()) return e;
        LOp o;
        o.gate = (int)i;
        o.gkind = x.kind;
        if (diag_kind(x.kind)) {
            // table over (targets, then controls); 1 where a control is 0
            o.kind = LOp::DIAG;
            o.k = k + x.n_ctrl;
            for (int j = 0; j < k; ++j) o.t[j] = pt[j];
            for (int j = 0; j < x.n_ctrl; ++j) o.t[k + j] = l2p[x.ctrl[j]];
            const int d = 1 << k;
            o.m.assign((size_t)1 << o.k, cd(1, 0));
            for (size_t idx = 0; idx < o.m.size(); ++idx) {
                const size_t cpart = idx >> k;
                if (cpart == (((size_t)1 << x.n_ctrl) - 1)) o.m[idx] = u[(idx & (d - 1)) * (d + 1)];
            }
            o.cphase = true;
            for (size_t idx = 0; idx + 1 < o.m.size(); ++idx) o.cphase = o.cphase && o.m[idx] == cd(1, 0);
        } else if (x.kind == QOPS_CX) {
            o.kind = LOp::ONEQ;
            o.k = 1;
            o.t[0] = pt[1];
            o.cmask = cm | (1ull << pt[0]);
            o.m = {cd(0), cd(1), cd(1), cd(0)};
        } else if (k == 1) {
            o.kind = LOp::ONEQ;
            o.k = 1;
            o.t[0] = pt[0];
            o.cmask = cm;
            o.m = u;
        } else {
            o.kind = LOp::DENSE;
            o.k = k;
            for (int j = 0; j < k; ++j) o.t[j] = pt[j];
            o.cmask = cm;
            o.m = u;
        }
        out.push_back(o);
    }
    return Err{};
}

// ---------------------------------------------------------------------------
// Merging (single-qubit merging and diagonal fusion), exact in FP64
// ---------------------------------------------------------------------------

static void mat2_mul(const std::vector<cd>& a, const std::vector<cd>& b, std::vector<cd>& out)
{
    out = {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3], a[2] * b[0] + a[3] * b[2], a[2] * b[1] + a[3] * b[3]};
}

static bool is_identity2(const std::vector<cd>& m)
{
    return std::abs(m[0] - 1.0) < 1e-14 && std::abs(m[1]) < 1e-14 && std::abs(m[2]) < 1e-14 &&
           std::abs(m[3] - 1.0) < 1e-14;
}

// X (later) merged into Y (earlier): Y <- X * Y for diagonal tables over bit sets.
static bool merge_diag(LOp& y, const LOp& x)
{
    uint64_t ub = 0;
    int bits[12];
    int nb = 0;
    for (int j = 0; j < y.k; ++j) {
        bits[nb++] = y.t[j];
        ub |= 1ull << y.t[j];
    }
    for (int j = 0; j < x.k; ++j)
        if (!(ub & (1ull << x.t[j]))) {
            if (nb >= 6) return false;
            bits[nb++] = x.t[j];
            ub |= 1ull << x.t[j];
        }
    std::vector<cd> tab((size_t)1 << nb);
    for (size_t idx = 0; idx < tab.size(); ++idx) {
        size_t iy = 0, ix = 0;
        for (int j = 0; j < y.k; ++j) iy |= ((idx >> j) & 1) << j;
        for (int j = 0; j < x.k; ++j) {
            int p = 0;
            while (bits[p] != x.t[j]) ++p;
            ix |= ((idx >> p) & 1) << j;
        }
        tab[idx] = y.m[iy] * x.m[ix];
    }
    y.k = nb;
    for (int j = 0; j < nb; ++j) y.t[j] = bits[j];
    y.m.swap(tab);
    y.nmerged += x.nmerged;
    y.cphase = true;
    for (size_t idx = 0; idx + 1 < y.m.size(); ++idx) y.cphase = y.cphase && y.m[idx] == cd(1, 0);
    return true;
}

// Left-multiplies the block matrix M (2^|Q| square, row-major, index bit i
// <-> physical bit Q[i]) by operation o embedded on the block's bits.
static void block_apply(std::vector<cd>& M, const std::vector<int>& Q, const LOp& o)
{
    const int nb = (int)Q.size();
    const uint32_t D = 1u << nb;
    auto bpos = [&](int phys) {
        for (int i = 0; i < nb; ++i)
            if (Q[i] == phys) return i;
        return -1;
    };
    uint32_t cm = 0;
    for (int b = 0; b < 64; ++b)
        if ((o.cmask >> b) & 1ull) cm |= 1u << bpos(b);
    if (o.kind == LOp::DIAG) {
        int tp[10];
        for (int j = 0; j < o.k; ++j) tp[j] = bpos(o.t[j]);
        for (uint32_t r = 0; r < D; ++r) {
            if ((r & cm) != cm) continue;
            uint32_t idx = 0;
            for (int j = 0; j < o.k; ++j) idx |= ((r >> tp[j]) & 1u) << j;
            const cd d = o.m[idx];
            for (uint32_t c = 0; c < D; ++c) M[(size_t)r * D + c] *= d;
        }
        return;
    }
    const int k = o.kind == LOp::PSWAP ? 2 : o.k;
    const uint32_t K = 1u << k;
    uint32_t off[64], tmask = 0;
    int tp[10];
    for (int j = 0; j < k; ++j) {
        tp[j] = bpos(o.t[j]);
        tmask |= 1u << tp[j];
    }
    for (uint32_t s = 0; s < K; ++s) {
        off[s] = 0;
        for (int j = 0; j < k; ++j)
            if (s & (1u << j)) off[s] |= 1u << tp[j];
    }
    std::vector<cd> in(K);
    for (uint32_t r0 = 0; r0 < D; ++r0) {
        if ((r0 & tmask) || (r0 & cm) != cm) continue;
        for (uint32_t c = 0; c < D; ++c) {
            for (uint32_t s = 0; s < K; ++s) in[s] = M[(size_t)(r0 | off[s]) * D + c];
            for (uint32_t r = 0; r < K; ++r) {
                cd acc = 0;
                for (uint32_t s = 0; s < K; ++s) acc += o.m[(size_t)r * K + s] * in[s];
                M[(size_t)(r0 | off[r]) * D + c] = acc;
            }
        }
    }
}

// Priced merging of dense blocks (the profile-guided choice of which gates
// to combine, Sec. III-C/D).  Cost of one block of k qubits in an LDS tile
// pass, in ms at 30 qubits: the marginal pass time per block.  Complex64:
// regressed from the per-pass times of a profiling run of Haar-block
// circuits (k = 2 on the vector ALU; k = 3 in the real embedding; k >= 4 in
// the three-product form; k = 5 in the 32x32x2 one).  Complex128: from
// circuits of 24 blocks of one width, the pass time above the memory phase
// (6.2 ms) per block.  Only the ratios matter: every cost scales with the
// state size.  Entry 1 is never used (merging takes blocks of 2 or more).
static const double kBlockCostC64[7] = {0.0, 0.30, 0.69, 0.94, 1.09, 1.69, 2.98};
static const double kBlockCostC128[7] = {0.0, 1.0, 1.74, 1.98, 2.20, 3.90, 5.98};

// Greedy, like fuse_blocks, over uncontrolled dense blocks of 2..6 qubits:
// a block absorbs a later one that commutes with every operation skipped in
// between when the union (<= 6 qubits) is priced below the two apart.  The
// merged matrix is the FP64 product in circuit order.
static void merge_dense_priced(std::vector<LOp>& ops, const double* cost)
{
    const size_t n = ops.size();
    const size_t window = 64;
    auto mergeable = [](const LOp& o) { return o.kind == LOp::DENSE && o.cmask == 0 && o.k >= 2 && !o.dead; };
    std::vector<char> placed(n, 0);
    std::vector<LOp> out;
    out.reserve(n);
    for (size_t first = 0; first < n; ++first) {
        if (placed[first]) continue;
        placed[first] = 1;
        const LOp& a = ops[first];
        if (!mergeable(a)) {
            out.push_back(a);
            continue;
        }
        uint64_t Qm = a.touch();
        std::vector<size_t> mem = {first};
        uint64_t skip_touch = 0, skip_nd = 0;
        const size_t stop = std::min(n, first + 1 + window);
        for (size_t j = first + 1; j < stop; ++j) {
            if (placed[j] || ops[j].dead) continue;
            const LOp& o = ops[j];
            if (o.kind == LOp::PSWAP) break;
            const uint64_t tj = o.touch(), nj = o.tmask();
            const bool commutes = (nj & skip_touch) == 0 && (tj & skip_nd) == 0;
            const int ku = __builtin_popcountll(Qm | tj);
            if (commutes && mergeable(o) && ku <= 6 &&
                cost[ku] < cost[__builtin_popcountll(Qm)] + cost[__builtin_popcountll(tj)]) {
                Qm |= tj;
                mem.push_back(j);
                placed[j] = 1;
            } else {
                skip_touch |= tj;
                skip_nd |= nj;
                if (__builtin_popcountll(skip_nd) >= 64) break;
            }
        }
        if (mem.size() == 1) {
            out.push_back(a);
            continue;
        }
        // the first block's qubit order first, then the new qubits in order
        std::vector<int> Q;
        for (int j = 0; j < a.k; ++j) Q.push_back(a.t[j]);
        for (size_t mi = 1; mi < mem.size(); ++mi)
            for (int j = 0; j < ops[mem[mi]].k; ++j)
                if (std::find(Q.begin(), Q.end(), ops[mem[mi]].t[j]) == Q.end()) Q.push_back(ops[mem[mi]].t[j]);
        const uint32_t D = 1u << Q.size();
        LOp f;
        f.kind = LOp::DENSE;
        f.k = (int)Q.size();
        for (int j = 0; j < f.k; ++j) f.t[j] = Q[j];
        f.cmask = 0;
        f.m.assign((size_t)D * D, cd(0));
        for (uint32_t i = 0; i < D; ++i) f.m[(size_t)i * D + i] = 1;
        f.gate = a.gate;
        f.gkind = QOPS_DENSE;
        f.nmerged = 0;
        for (size_t j : mem) {
            block_apply(f.m, Q, ops[j]);
            f.nmerged += ops[j].nmerged;
        }
        out.push_back(std::move(f));
    }
    ops.swap(out);
}

// k-qubit block fusion: ops whose bits (targets, controls, table bits) fit a
// common set of at most kmax physical bits become one dense 2^k x 2^k block,
// the FP64 product of the ops embedded on that set.  Each block opens with
// the first op not yet placed and scans ahead, taking ops that fit and
// commute with every op skipped so far (the same rule as pass packing).
// Blocks of a single op, and blocks of diagonals only, are kept as they are.
static void fuse_blocks(std::vector<LOp>& ops, int kmax)
{
    if (kmax < 2) return;
    const size_t n = ops.size();
    const size_t window = 64;
    std::vector<char> placed(n, 0);
    std::vector<LOp> out;
    out.reserve(n);
    for (size_t first = 0; first < n; ++first) {
        if (placed[first]) continue;
        placed[first] = 1;
        const LOp& a = ops[first];
        if (a.dead) continue;
        if (a.kind == LOp::PSWAP || __builtin_popcountll(a.touch()) > kmax) {
            out.push_back(a);
            continue;
        }
        uint64_t Qm = a.touch();
        std::vector<size_t> mem = {first};
        uint64_t skip_touch = 0, skip_nd = 0;
        const size_t stop = std::min(n, first + 1 + window);
        for (size_t j = first + 1; j < stop; ++j) {
            if (placed[j] || ops[j].dead) continue;
            const LOp& o = ops[j];
            if (o.kind == LOp::PSWAP) break;
            const uint64_t tj = o.touch(), nj = o.tmask();
            const bool commutes = (nj & skip_touch) == 0 && (tj & skip_nd) == 0;
            if (commutes && __builtin_popcountll(Qm | tj) <= kmax) {
                Qm |= tj;
                mem.push_back(j);
                placed[j] = 1;
            } else {
                skip_touch |= tj;
                skip_nd |= nj;
            }
        }
        bool all_diag = true;
        for (size_t j : mem) all_diag = all_diag && ops[j].kind == LOp::DIAG;
        if (mem.size() == 1 || all_diag) {
            for (size_t j : mem) out.push_back(ops[j]);
            continue;
        }
        std::vector<int> Q;
        for (int b = 0; b < 64; ++b)
            if ((Qm >> b) & 1ull) Q.push_back(b);
        const uint32_t D = 1u << Q.size();
        LOp f;
        f.kind = LOp::DENSE;
        f.k = (int)Q.size();
        for (int j = 0; j < f.k; ++j) f.t[j] = Q[j];
        f.cmask = 0;
        f.m.assign((size_t)D * D, cd(0));
        for (uint32_t i = 0; i < D; ++i) f.m[(size_t)i * D + i] = 1;
        f.gate = a.gate;
        f.gkind = QOPS_DENSE;
        f.nmerged = 0;
        for (size_t j : mem) {
            block_apply(f.m, Q, ops[j]);
            f.nmerged += ops[j].nmerged;
        }
        out.push_back(std::move(f));
    }
    ops.swap(out);
}

static void merge_ops(std::vector<LOp>& in, std::vector<LOp>& out)
{
    const int kScan = 96;
    out.clear();
    out.reserve(in.size());
    for (LOp& x : in) {
        bool merged = false;
        if (x.kind == LOp::ONEQ) {
            const uint64_t tb = 1ull << x.t[0];
            for (int j = (int)out.size() - 1, c = 0; j >= 0 && c < kScan; --j, ++c) {
                LOp& y = out[j];
                if (y.dead) continue;
                if (y.kind == LOp::ONEQ && y.t[0] == x.t[0] && y.cmask == x.cmask) {
                    std::vector<cd> p;
                    mat2_mul(x.m, y.m, p);
                    y.m.swap(p);
                    y.nmerged += x.nmerged;
                    if (is_identity2(y.m)) y.dead = true;
                    merged = true;
                    break;
                }
                if (x.cmask == 0 && y.kind == LOp::DIAG && y.k == 1 && y.t[0] == x.t[0]) {
                    // U * diag(d): the diagonal joins the 2x2
                    std::vector<cd> p = {x.m[0] * y.m[0], x.m[1] * y.m[1], x.m[2] * y.m[0], x.m[3] * y.m[1]};
                    y.kind = LOp::ONEQ;
                    y.k = 1;
                    y.cmask = 0;
                    y.cphase = false;
                    y.m.swap(p);
                    y.nmerged += x.nmerged;
                    y.gkind = x.gkind;
                    merged = true;
                    break;
                }
                if (y.touch() & tb) break;
                if (y.tmask() & x.cmask) break;
            }
        } else if (x.kind == LOp::DIAG) {
            uint64_t xb = 0;
            for (int j = 0; j < x.k; ++j) xb |= 1ull << x.t[j];
            // a one-bit diagonal prefers the 2x2 on its qubit; otherwise the
            // nearest diagonal table with room takes it
            int diag_cand = -1;
            for (int j = (int)out.size() - 1, c = 0; j >= 0 && c < kScan; --j, ++c) {
                LOp& y = out[j];
                if (y.dead) continue;
                // controlled phases merge only with a controlled phase on the
                // same bits (the product is again one); general tables merge
                // with general tables
                bool same_bits = y.kind == LOp::DIAG && y.k == x.k;
                for (int b = 0; same_bits && b < x.k; ++b) same_bits = y.t[b] == x.t[b];
                const bool compatible = (!x.cphase && !y.cphase) || (x.cphase && y.cphase && same_bits);
                if (y.kind == LOp::DIAG && diag_cand < 0 && compatible) {
                    LOp probe = y;
                    if (merge_diag(probe, x)) {
                        diag_cand = j;
                        if (x.k != 1) break;
                    }
                }
                if (x.k == 1 && y.kind == LOp::ONEQ && y.cmask == 0 && y.t[0] == x.t[0]) {
                    std::vector<cd> p = {x.m[0] * y.m[0], x.m[0] * y.m[1], x.m[1] * y.m[2], x.m[1] * y.m[3]};
                    y.m.swap(p);
                    y.nmerged += x.nmerged;
                    merged = true;
                    break;
                }
                if (y.tmask() & xb) break;
            }
            if (!merged && diag_cand >= 0) merged = merge_diag(out[diag_cand], x);
        }
        if (!merged) out.push_back(x);
    }
    std::vector<LOp> alive;
    alive.reserve(out.size());
    for (LOp& o : out)
        if (!o.dead) alive.push_back(std::move(o));
    out.swap(alive);
}

// ---------------------------------------------------------------------------
// Device program emission
// ---------------------------------------------------------------------------

static int push_coef(Plan& p, const std::vector<cd>& m)
{
    const int off = (int)p.coef.size();
    for (const cd& v : m) {
        p.coef.push_back(v.real());
        p.coef.push_back(v.imag());
    }
    return off;
}

// A fragments of the real embedding M (rows/cols interleaved re,im) for the
// 16x16x4 matrix-core layout: A[(rb*KS + ks)*64 + l] = M[16 rb + rho(l%16)][4 ks + l/16].
// The f32 instruction returns row 4*(l/16)+i of its result in lane l,
// register i; the f64 one returns row l/16 + 4*i.  For f64 the A rows are
// permuted (rho(x) = 4*(x%4) + x/4) so that both land in the same place and
// the kernel's write-back is shared.
// Coefficients of a matrix-core block: k = 3 uses the real embedding
// (2^(k+1) square, 4^(k+1) values), k >= 4 Gauss's three-product form (the
// real part, the imaginary part and their sum of each k-step fragment,
// 3 * 4^k values).
static size_t mfma_coef_count(int k) { return k >= 4 ? size_t(3) << (2 * k) : size_t(1) << (2 * (k + 1)); }

static int push_mfma_coef(Plan& p, const std::vector<cd>& u, int k)
{
    const int d = 1 << k, D = 2 * d;
    if (k >= 4) {
        // fragment (rb, ks, m), lane l: row 16 rb + x (x = l % 16, permuted for
        // the FP64 result layout), column 4 ks + l / 16, of A (m = 0), B (1) or
        // A + B (2), composed in FP64
        const int KS = d / 4, RB = d / 16;
        const int off = (int)p.coef.size();
        for (int rb = 0; rb < RB; ++rb)
            for (int ks = 0; ks < KS; ++ks)
                for (int m = 0; m < 3; ++m)
                    for (int l = 0; l < 64; ++l) {
                        const int x = l & 15;
                        const int row = p.prec == QOPS_C64 ? x : 4 * (x & 3) + (x >> 2);
                        const cd v = u[(size_t)(16 * rb + row) * d + (4 * ks + (l >> 4))];
                        p.coef.push_back(m == 0 ? v.real() : (m == 1 ? v.imag() : v.real() + v.imag()));
                    }
        return off;
    }
    const int KS = D / 4, RB = D / 16;
    auto Mre = [&](int r, int c) -> double {
        const cd v = u[(size_t)(r >> 1) * d + (c >> 1)];
        const int pr = r & 1, pc = c & 1;
        if (pr == 0 && pc == 0) return v.real();
        if (pr == 0 && pc == 1) return -v.imag();
        if (pr == 1 && pc == 0) return v.imag();
        return v.real();
    };
    const int off = (int)p.coef.size();
    for (int rb = 0; rb < RB; ++rb)
        for (int ks = 0; ks < KS; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int x = l & 15;
                const int row = p.prec == QOPS_C64 ? x : 4 * (x & 3) + (x >> 2);
                p.coef.push_back(Mre(16 * rb + row, 4 * ks + (l >> 4)));
            }
    return off;
}

// Coefficients of a 5- or 6-qubit block in the 32x32x2 three-product form
// (complex64, largest LDS tile): fragment (rb, ks, m), lane l holds row
// 32 rb + l % 32, column 2 ks + l / 32 of A (m = 0), B (1) or A + B (2);
// 3 * 4^k values, as in the 16x16x4 form.
static int push_mfma_coef_wide(Plan& p, const std::vector<cd>& u, int k)
{
    const int d = 1 << k, KS = d / 2, RB = d / 32;
    const int off = (int)p.coef.size();
    for (int rb = 0; rb < RB; ++rb)
        for (int ks = 0; ks < KS; ++ks)
            for (int m = 0; m < 3; ++m)
                for (int l = 0; l < 64; ++l) {
                    const cd v = u[(size_t)(32 * rb + (l & 31)) * d + (2 * ks + (l >> 5))];
                    p.coef.push_back(m == 0 ? v.real() : (m == 1 ? v.imag() : v.real() + v.imag()));
                }
    return off;
}

static void fill_runs(int n, int fixed, const std::vector<int>& up, PassHdr& h)
{
    std::vector<bool> intile(n, false);
    for (int b = 0; b < std::min(n, fixed); ++b) intile[b] = true;
    for (int u : up) intile[u] = true;
    h.nruns = 0;
    int g = 0;
    for (int b = 0; b < n;) {
        if (intile[b]) {
            ++b;
            continue;
        }
        int e = b;
        while (e < n && !intile[e]) ++e;
        h.run_start[h.nruns] = b;
        h.run_len[h.nruns] = e - b;
        h.run_gshift[h.nruns] = g;
        g += e - b;
        ++h.nruns;
        b = e;
    }
}

// Vector-ALU dense blocks are compiled for k <= 4 (c64) / k <= 3 (c128);
// matrix-core blocks need k >= 3 and at least 16 groups (L >= k + 4).
static bool valu_ok(const Plan& p, int k) { return p.prec == 0 ? k <= 4 : k <= 3; }
// the matrix-core stage is compiled for tiles of up to 2^13 (c64) / 2^12
// (c128) amplitudes
static bool mfma_possible(int k, int L) { return k >= 3 && L >= k + 4; }
static bool use_mfma_for(const Plan& p, int k, int L)
{
    if (!mfma_possible(k, L)) return false;
    if (!valu_ok(p, k)) return true;
    return p.par.use_mfma != 0;
}
static bool lds_capable(const Plan& p, const LOp& o, int L)
{
    if (o.kind == LOp::DIAG || o.kind == LOp::ONEQ || o.kind == LOp::PSWAP) return true;
    return valu_ok(p, o.k) || mfma_possible(o.k, L);
}

// LDS-resident ops (tile LDS, whole-state LDS and sweep share the encoding;
// `tpos(phys)` maps a physical bit to a tile position or -1 if outside).
// Column positions of a matrix-core op: a column is one group of 2^k
// amplitudes (one value of the L-k free tile positions); the 16 columns a
// wave reads at once differ in four free positions (c_lane), the column
// block number fills the rest (c_wave).  The LDS swizzle folds tile
// positions 5..9 onto 0..4, so position p falls in bank class p (p < 5),
// p - 5 (p < 10) or none.  The 32 lanes of half a wave read 16 columns times
// the two values of the op's matrix bit 0, and hit distinct banks when those
// five positions have distinct classes.  Writes go the same way with the
// result rows: half a wave writes 16 columns times the two values of matrix
// bit 1 (real embedding, k = 3) or bit 2 (three-product form, k >= 4).  The
// op's targets for these two matrix bits are chosen so that the columns can
// avoid both classes (best when the two share one), then the columns take
// distinct classes.
static int bank_class(int tp) { return tp < 5 ? tp : (tp < 10 ? tp - 5 : -1); }

// Matrix bit whose two values share half a wave in the write-back.
static int write_bit(int k) { return k >= 4 ? 2 : 1; }

static uint32_t class_bit(int tp)
{
    const int r = bank_class(tp);
    return r >= 0 ? 1u << r : 0u;
}

// Picks up to four free positions (not in opm) with distinct classes outside
// the classes in `avoid` (a bit mask of classes), then fills up to four.
static void pick_columns(uint32_t opm, int L, uint32_t avoid, uint32_t& used)
{
    uint32_t taken = 0;
    used = 0;
    int got = 0;
    for (int tp = 0; tp < L && got < 4; ++tp) {
        if (opm & (1u << tp)) continue;
        const uint32_t c = class_bit(tp);
        if (c && !(avoid & c) && !(taken & c)) {
            taken |= c;
            used |= 1u << tp;
            ++got;
        }
    }
    for (int tp = 0; tp < L && __builtin_popcount(used) < 4; ++tp)
        if (!(opm & (1u << tp)) && !(used & (1u << tp))) used |= 1u << tp;
}

// Distinct bank classes among the column positions and one more position.
static int distinct_classes(uint32_t used, int extra)
{
    uint32_t m = class_bit(extra);
    for (int tp = 0; tp < 32; ++tp)
        if (used & (1u << tp)) m |= class_bit(tp);
    return __builtin_popcount(m);
}

// Columns for an op whose read and write bits sit at tile positions t0, tw:
// avoiding both classes, or only one of them (four free classes for the
// columns can beat three); returns the distinct classes reached, reads plus
// writes (ties keep the earlier choice).
static int best_columns(uint32_t opm, int L, int t0, int tw, uint32_t& used)
{
    const uint32_t masks[3] = {class_bit(t0) | class_bit(tw), class_bit(t0), class_bit(tw)};
    int best = -1;
    for (uint32_t av : masks) {
        uint32_t u;
        pick_columns(opm, L, av, u);
        const int sc = distinct_classes(u, t0) + distinct_classes(u, tw);
        if (sc > best) {
            best = sc;
            used = u;
        }
    }
    return best;
}

static void set_mfma_columns(DevOp& d, int k, int L)
{
    uint32_t opm = 0;
    for (int j = 0; j < k; ++j) opm |= 1u << d.pos[j];
    uint32_t used = 0;
    best_columns(opm, L, d.pos[0], d.pos[write_bit(k)], used);
    const uint32_t all = (L >= 32 ? ~0u : ((1u << L) - 1u));
    d.c_lane = used;
    d.c_wave = all & ~opm & ~used;
}

// Columns of a block in the 32x32x2 form: half a wave reads (and writes) one
// matrix index of 32 columns, which differ in the five positions of c_lane;
// they hit 32 distinct banks when those positions cover the five bank
// classes.  Positions are taken class by class, then filled up to five.
static void set_mfma_columns_wide(DevOp& d, int k, int L)
{
    uint32_t opm = 0;
    for (int j = 0; j < k; ++j) opm |= 1u << d.pos[j];
    uint32_t used = 0, taken = 0;
    for (int tp = 0; tp < L; ++tp) {
        const uint32_t c = class_bit(tp);
        if ((opm & (1u << tp)) || !c || (taken & c)) continue;
        taken |= c;
        used |= 1u << tp;
    }
    for (int tp = 0; tp < L && __builtin_popcount(used) < 5; ++tp)
        if (!(opm & (1u << tp)) && !(used & (1u << tp))) used |= 1u << tp;
    const uint32_t all = (L >= 32 ? ~0u : ((1u << L) - 1u));
    d.c_lane = used;
    d.c_wave = all & ~opm & ~used;
    d.c_reg = QOPS_MFMA_WIDE;
}

// Which targets become matrix bit 0 (reads) and the write bit: the pair that
// reaches the most distinct classes (ties keep the lower indices).
static void best_bank_bits(const int* tp, int k, int L, int& j0, int& jw)
{
    uint32_t opm = 0;
    for (int j = 0; j < k; ++j) opm |= 1u << tp[j];
    int score = -1;
    j0 = 0;
    jw = write_bit(k);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            if (a == b) continue;
            uint32_t used;
            const int sc = best_columns(opm, L, tp[a], tp[b], used);
            if (sc > score) {
                score = sc;
                j0 = a;
                jw = b;
            }
        }
}

// Exchanges matrix bits p and q of a 2^k x 2^k matrix (and the targets).
static void swap_matrix_bits(std::vector<cd>& m, int* t, int k, int p, int q)
{
    if (p == q) return;
    const int d = 1 << k;
    auto sw = [&](int x) {
        const int bp = (x >> p) & 1, bq = (x >> q) & 1;
        return (x & ~(1 << p) & ~(1 << q)) | (bp << q) | (bq << p);
    };
    std::vector<cd> r((size_t)d * d);
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) r[(size_t)sw(a) * d + sw(b)] = m[(size_t)a * d + b];
    m.swap(r);
    std::swap(t[p], t[q]);
}

// Moves targets j0 and jw (j0 != jw) to matrix bits 0 and the write bit.
static void place_bank_bits(std::vector<cd>& m, int* t, int* tp, int k, int j0, int jw)
{
    const int w = write_bit(k);
    swap_matrix_bits(m, t, k, 0, j0);
    std::swap(tp[0], tp[j0]);
    if (jw == 0) jw = j0;   // that target now sits where the bit-0 one was
    swap_matrix_bits(m, t, k, w, jw);
    std::swap(tp[w], tp[jw]);
}

template <typename F>
static void emit_lds_op(Plan& p, const LOp& o, int L, F tpos, PassPlan& pp, bool wide_ok = false)
{
    DevOp d;
    std::memset(&d, 0, sizeof(d));
    if (o.kind == LOp::DIAG) {
        d.type = OP_DIAG_LDS;
        d.a = o.k;
        for (int j = 0; j < o.k; ++j) {
            const int tp = tpos(o.t[j]);
            d.pos[j] = tp >= 0 ? enc_src(SRC_LANE, tp) : enc_src(SRC_GLOB, o.t[j]);
        }
        d.coef = push_coef(p, o.m);
        pp.n_diag_ops++;
    } else {
        std::vector<cd> m = o.m;
        int k = o.k;
        int t[6];
        for (int j = 0; j < k; ++j) t[j] = o.t[j];
        if (o.kind == LOp::PSWAP) {
            k = 2;
            m.assign(16, cd(0));
            m[0] = 1;
            m[1 * 4 + 2] = 1;
            m[2 * 4 + 1] = 1;
            m[15] = 1;
        }
        const bool wide = wide_ok && o.kind == LOp::DENSE && k == 5 && use_mfma_for(p, k, L);
        if (o.kind == LOp::DENSE && use_mfma_for(p, k, L) && !wide) {
            int tp[6];
            for (int j = 0; j < k; ++j) tp[j] = tpos(t[j]);
            int j0 = 0, jw = 1;
            best_bank_bits(tp, k, L, j0, jw);
            place_bank_bits(m, t, tp, k, j0, jw);
        }
        for (int j = 0; j < k; ++j) d.pos[j] = tpos(t[j]);
        for (int b = 0; b < 64; ++b)
            if (o.cmask & (1ull << b)) {
                const int tp = tpos(b);
                if (tp >= 0) d.c_tile |= 1u << tp;
                else d.c_glob |= 1ull << b;
            }
        d.a = k;
        if (use_mfma_for(p, k, L)) {
            d.type = OP_MFMA;
            pp.n_mfma++;
            if (wide) {
                d.coef = push_mfma_coef_wide(p, m, k);
                set_mfma_columns_wide(d, k, L);
            } else {
                d.coef = push_mfma_coef(p, m, k);
                set_mfma_columns(d, k, L);
            }
        } else {
            d.type = OP_DENSE_LDS;
            d.coef = push_coef(p, m);
            if (k == 1) pp.n_reg_ops++;
            else pp.n_dense++;
        }
        pp.max_k = std::max(pp.max_k, k);
        pp.flops += 8.0 * (double)(1 << k) * std::ldexp(1.0, p.n);
    }
    p.dops.push_back(d);
}

// Register-tile pass: assigns register/wave bits per stage and encodes ops.
static void emit_tile_reg(Plan& p, PassPlan& pp)
{
    const int R = pp.R, W = pp.W, U = R + W;
    const std::vector<int>& up = pp.up;
    auto upos = [&](int phys) {
        for (int u = 0; u < U; ++u)
            if (up[u] == phys) return u;
        return -1;
    };
    // sequence of upper positions needed in registers, in op order
    std::vector<int> need;
    for (int li : pp.lop) {
        const LOp& o = p.lops[li];
        if (o.kind == LOp::ONEQ && o.t[0] >= 6) need.push_back(upos(o.t[0]));
        else need.push_back(-1);
    }
    auto choose = [&](size_t from, const std::vector<int>& keep) {
        std::vector<int> regs;
        for (size_t i = from; i < need.size() && (int)regs.size() < R; ++i)
            if (need[i] >= 0 && std::find(regs.begin(), regs.end(), need[i]) == regs.end()) regs.push_back(need[i]);
        for (int u : keep)
            if ((int)regs.size() < R && std::find(regs.begin(), regs.end(), u) == regs.end()) regs.push_back(u);
        for (int u = 0; u < U && (int)regs.size() < R; ++u)
            if (std::find(regs.begin(), regs.end(), u) == regs.end()) regs.push_back(u);
        return regs;
    };
    auto mapword = [&](const std::vector<int>& regs) {
        uint32_t m = 0;
        int i = 0;
        for (int u : regs) m |= (uint32_t)u << (4 * i++);
        for (int u = 0; u < U; ++u)
            if (std::find(regs.begin(), regs.end(), u) == regs.end()) m |= (uint32_t)u << (4 * i++);
        return m;
    };
    std::vector<int> regs = choose(0, {});
    uint32_t map = mapword(regs);
    PassHdr h;
    std::memset(&h, 0, sizeof(h));
    h.hoist = -1;
    h.n = p.n;
    h.L = pp.L;
    h.nup = U;
    h.map0 = map;
    for (int u = 0; u < U; ++u) h.up_phys[u] = up[u];
    fill_runs(p.n, 6, up, h);
    h.op0 = (int)p.dops.size();
    auto regbit = [&](int u) {
        for (int b = 0; b < R; ++b)
            if (map_get(map, b) == u) return b;
        return -1;
    };
    auto wavebit = [&](int u) {
        for (int w = 0; w < W; ++w)
            if (map_get(map, R + w) == u) return w;
        return -1;
    };
    for (size_t i = 0; i < pp.lop.size(); ++i) {
        const LOp& o = p.lops[pp.lop[i]];
        if (need[i] >= 0 && regbit(need[i]) < 0) {
            regs = choose(i, regs);
            map = mapword(regs);
            DevOp r;
            std::memset(&r, 0, sizeof(r));
            r.type = OP_REMAP;
            r.b = (int32_t)map;
            p.dops.push_back(r);
            pp.n_remaps++;
        }
        DevOp d;
        std::memset(&d, 0, sizeof(d));
        auto enc_ctrl = [&](uint64_t cm) {
            for (int b = 0; b < 64; ++b) {
                if (!(cm & (1ull << b))) continue;
                if (b < 6) {
                    d.c_lane |= 1u << b;
                    continue;
                }
                const int u = upos(b);
                if (u < 0) {
                    d.c_glob |= 1ull << b;
                } else if (regbit(u) >= 0) {
                    d.c_reg |= 1u << regbit(u);
                } else {
                    d.c_wave |= 1u << wavebit(u);
                }
            }
        };
        if (o.kind == LOp::ONEQ) {
            if (o.t[0] < 6) {
                d.type = OP_1Q_LANE;
                d.a = o.t[0];
                pp.n_lane_ops++;
            } else {
                d.type = OP_1Q_REG;
                d.a = regbit(upos(o.t[0]));
                pp.n_reg_ops++;
            }
            enc_ctrl(o.cmask);
            d.coef = push_coef(p, o.m);
            const bool is_x = o.m[0] == cd(0) && o.m[1] == cd(1) && o.m[2] == cd(1) && o.m[3] == cd(0);
            d.b = is_x ? 1 : 0;
            if (!is_x) pp.flops += 16.0 * std::ldexp(1.0, p.n - __builtin_popcountll(o.cmask));
        } else if (o.cphase) {
            // phase on the all-ones pattern of the table bits: a control mask
            d.type = OP_CPHASE;
            uint64_t bm = 0;
            for (int j = 0; j < o.k; ++j) bm |= 1ull << o.t[j];
            enc_ctrl(bm);
            const cd ph = o.m.back();
            d.coef = push_coef(p, {ph});
            d.b = ph == cd(-1, 0) ? 1 : 0;
            pp.n_diag_ops++;
            pp.flops += 6.0 * std::ldexp(1.0, p.n - o.k);
        } else {   // DIAG
            d.type = OP_DIAG;
            d.a = o.k;
            for (int j = 0; j < o.k; ++j) {
                const int b = o.t[j];
                if (b < 6) {
                    d.pos[j] = enc_src(SRC_LANE, b);
                    continue;
                }
                const int u = upos(b);
                if (u < 0) d.pos[j] = enc_src(SRC_GLOB, b);
                else if (regbit(u) >= 0) d.pos[j] = enc_src(SRC_REG, regbit(u));
                else d.pos[j] = enc_src(SRC_WAVE, wavebit(u));
            }
            d.coef = push_coef(p, o.m);
            pp.n_diag_ops++;
            pp.flops += 6.0 * std::ldexp(1.0, p.n);
        }
        p.dops.push_back(d);
    }
    h.nops = (int)p.dops.size() - h.op0;
    h.lds_bytes = W > 0 ? (1 << pp.L) * (p.prec == 0 ? 8 : 16) : 0;
    pp.op0 = h.op0;
    pp.nops = h.nops;
    pp.hdr = (int)p.hdrs.size();
    p.hdrs.push_back(h);
}

// Bytes of coefficients an LDS tile pass stages in LDS for an op (matrix-core
// fragments and diagonal tables); 0 for ops that read theirs with scalar loads.
static size_t staged_bytes(const Plan& p, const LOp& o, int L)
{
    const size_t sz = p.prec == 0 ? 4 : 8;
    if (o.kind == LOp::DIAG) return (size_t(2) << o.k) * sz;
    const int k = o.kind == LOp::PSWAP ? 2 : o.k;
    if (o.kind == LOp::DENSE && use_mfma_for(p, k, L)) return mfma_coef_count(k) * sz;
    return (size_t(2) << (2 * k)) * sz;   // 2^k x 2^k complex for the vector ALU
}

// The matrix-core block of a complex64 LDS pass whose fragments stay in
// registers: the first of the widest blocks of 5 or 6 qubits; -1 if none.
static int hoist_choice(const Plan& p, int op0, int nops)
{
    if (p.prec != 0) return -1;
    int at = -1, best = 4;
    for (int i = op0; i < op0 + nops; ++i)
        if (p.dops[i].type == OP_MFMA && p.dops[i].a > best) {
            best = p.dops[i].a;
            at = i - op0;
        }
    return at;
}

// LDS of one work-group of the LDS tile kernel: complex64 passes run two
// work-groups per CU (the kernel is register-bounded for it), complex128 one
static size_t lds_budget(int prec) { return prec == 0 ? QOPS_LDS_TILE_BYTES_C64 : QOPS_LDS_TILE_BYTES_C128; }

static void emit_tile_lds(Plan& p, PassPlan& pp)
{
    PassHdr h;
    std::memset(&h, 0, sizeof(h));
    h.n = p.n;
    h.L = pp.L;
    h.nup = (int)pp.up.size();
    for (int u = 0; u < h.nup; ++u) h.up_phys[u] = pp.up[u];
    fill_runs(p.n, QOPS_LDS_FIXED_BITS, pp.up, h);
    h.op0 = (int)p.dops.size();
    auto tpos = [&](int phys) {
        if (phys < QOPS_LDS_FIXED_BITS) return phys;
        for (int u = 0; u < h.nup; ++u)
            if (pp.up[u] == phys) return QOPS_LDS_FIXED_BITS + u;
        return -1;
    };
    // complex64 passes on the largest tile run their 5-qubit blocks in the
    // 32x32x2 form
    const bool wide_ok = p.prec == 0 && pp.L == 13;
    for (int li : pp.lop) emit_lds_op(p, p.lops[li], pp.L, tpos, pp, wide_ok);
    h.nops = (int)p.dops.size() - h.op0;
    // stage the per-lane coefficients (matrix-core fragments, diagonal
    // tables) contiguously, as far as they fit next to the tile in LDS
    const size_t sz = p.prec == 0 ? 4 : 8;
    const size_t tile_bytes = (size_t(1) << pp.L) * 2 * sz;
    size_t room = lds_budget(p.prec) > tile_bytes ? (lds_budget(p.prec) - tile_bytes) / sz : 0;
    // complex64: the widest matrix-core block of 5 or 6 qubits keeps its
    // fragments in registers across the pass's tiles (loaded once, before
    // the tile loop, so it needs no staging); every other op is staged (the
    // packer keeps them within the LDS budget)
    h.hoist = hoist_choice(p, h.op0, h.nops);
    h.coef_src = (int)p.coef.size();
    int staged = 0;
    for (int i = h.op0; i < h.op0 + h.nops; ++i) {
        DevOp& d = p.dops[i];
        d.b = 0;
        if (d.type != OP_MFMA && d.type != OP_DIAG_LDS && d.type != OP_DENSE_LDS) continue;
        if (i - h.op0 == h.hoist) continue;
        size_t cnt;
        if (d.type == OP_MFMA) cnt = mfma_coef_count(d.a);
        else if (d.type == OP_DENSE_LDS) cnt = size_t(2) << (2 * d.a);
        else cnt = size_t(2) << d.a;
        if (cnt > room) continue;
        const int off = (int)p.coef.size();
        p.coef.insert(p.coef.end(), p.coef.begin() + d.coef, p.coef.begin() + d.coef + cnt);
        d.coef = off - h.coef_src;
        d.b = 1;
        room -= cnt;
        staged += (int)cnt;
    }
    h.coef_n = staged;
    h.lds_bytes = (int)(tile_bytes + (size_t)staged * sz);
    pp.op0 = h.op0;
    pp.nops = h.nops;
    pp.hdr = (int)p.hdrs.size();
    p.hdrs.push_back(h);
}

static void emit_state_lds(Plan& p, PassPlan& pp)
{
    pp.op0 = (int)p.dops.size();
    auto tpos = [&](int phys) { return phys; };
    for (int li : pp.lop) emit_lds_op(p, p.lops[li], p.n, tpos, pp);
    pp.nops = (int)p.dops.size() - pp.op0;
}

static void emit_sweep(Plan& p, PassPlan& pp)
{
    const LOp& o = p.lops[pp.lop[0]];
    DevOp d;
    std::memset(&d, 0, sizeof(d));
    if (o.kind == LOp::DIAG) {
        d.type = OP_DIAG_LDS;
        d.a = o.k;
        for (int j = 0; j < o.k; ++j) d.pos[j] = o.t[j];   // raw physical bits
        d.coef = push_coef(p, o.m);
        pp.n_diag_ops = 1;
    } else {
        d.type = OP_DENSE_LDS;
        d.a = o.k;
        for (int j = 0; j < o.k; ++j) d.pos[j] = o.t[j];
        d.c_glob = o.cmask;
        d.coef = push_coef(p, o.m);
        pp.max_k = o.k;
        if (o.k == 1) pp.n_reg_ops = 1;
        else pp.n_dense = 1;
        pp.flops = 8.0 * (double)(1 << o.k) * std::ldexp(1.0, p.n - __builtin_popcountll(o.cmask));
    }
    pp.op0 = (int)p.dops.size();
    pp.nops = 1;
    p.dops.push_back(d);
}

// ---------------------------------------------------------------------------
// Packing
// ---------------------------------------------------------------------------

static size_t staged_bytes(const Plan& p, const LOp& o, int L);
static size_t lds_budget(int prec);

static void pick_reg_variant(int n, int prec, int want_up, int& R, int& W)
{
    // available variants: R in {4,5}, W in {0,1,2}
    int U = std::min(want_up, n - 6);
    U = std::max(4, std::min(U, 7));
    R = prec == 0 ? std::min(5, U) : std::min(4, U);
    W = U - R;
    if (W > 2) {
        W = 2;
        R = U - W;
        if (R > 5) R = 5;
    }
}

static void finish_pass(Plan& p, PassPlan& pp, uint64_t upmask, bool dense)
{
    const int n = p.n;
    const double sz = p.prec == 0 ? 8.0 : 16.0;
    int cap, fixed;
    if (dense) {
        pp.type = PASS_TILE_LDS;
        fixed = QOPS_LDS_FIXED_BITS;
        cap = std::min(p.par.L_lds, n) - fixed;
    } else {
        pp.type = PASS_TILE_REG;
        fixed = 6;
        cap = pp.R + pp.W;
    }
    // the bits the ops need, then the lowest free bits (longer contiguous
    // runs in memory)
    pp.up.clear();
    for (int b = fixed; b < n; ++b)
        if (upmask & (1ull << b)) pp.up.push_back(b);
    for (int b = fixed; b < n && (int)pp.up.size() < cap; ++b)
        if (!(upmask & (1ull << b))) pp.up.push_back(b);
    std::sort(pp.up.begin(), pp.up.end());
    pp.L = fixed + (int)pp.up.size();
    pp.bytes_alg = 2.0 * std::ldexp(1.0, n) * sz;
    if (pp.type == PASS_TILE_LDS) emit_tile_lds(p, pp);
    else emit_tile_reg(p, pp);
}

static void pack(Plan& p)
{
    const int n = p.n;
    const double sz = p.prec == 0 ? 8.0 : 16.0;
    const double state_bytes = std::ldexp(1.0, n) * sz;
    p.passes.clear();
    p.hdrs.clear();
    p.dops.clear();
    p.coef.clear();
    if (p.par.mode == QOPS_PLAN_GATEWISE) {
        for (size_t i = 0; i < p.lops.size(); ++i) {
            PassPlan pp;
            const LOp& o = p.lops[i];
            if (o.kind == LOp::PSWAP) {
                pp.type = PASS_SWAP_BITS;
                pp.swap_a = o.t[0];
                pp.swap_b = o.t[1];
                pp.bytes_alg = state_bytes;
                pp.lop.push_back((int)i);
            } else {
                pp.type = PASS_SWEEP;
                pp.lop.push_back((int)i);
                emit_sweep(p, pp);
                const int c = o.kind == LOp::DIAG ? 0 : __builtin_popcountll(o.cmask);
                pp.bytes_alg = 2.0 * state_bytes * std::ldexp(1.0, -c);
            }
            p.passes.push_back(pp);
        }
        return;
    }
    if (n <= p.par.state_lds_max_n) {
        // whole state in LDS; blocks the LDS kernel cannot take run as sweeps
        PassPlan pp;
        auto flush_state = [&]() {
            if (pp.lop.empty()) return;
            pp.type = PASS_STATE_LDS;
            pp.L = n;
            emit_state_lds(p, pp);
            pp.bytes_alg = 2.0 * state_bytes;
            p.passes.push_back(pp);
            pp = PassPlan();
        };
        for (size_t i = 0; i < p.lops.size(); ++i) {
            if (lds_capable(p, p.lops[i], n)) {
                pp.lop.push_back((int)i);
                continue;
            }
            flush_state();
            PassPlan sw;
            sw.type = PASS_SWEEP;
            sw.lop.push_back((int)i);
            emit_sweep(p, sw);
            sw.bytes_alg = 2.0 * state_bytes;
            p.passes.push_back(sw);
        }
        flush_state();
        return;
    }
    int R, W;
    pick_reg_variant(n, p.prec, p.par.R + p.par.W, R, W);
    const int cap_reg = R + W;
    const int cap_lds = std::min(p.par.L_lds, n) - QOPS_LDS_FIXED_BITS;
    PassPlan cur;
    cur.R = R;
    cur.W = W;
    uint64_t S = 0;           // needed bits beyond a register tile's six fixed ones
    uint64_t S4 = 0;          //   and beyond an LDS tile's fixed ones
    bool dense = false;
    size_t staged = 0;        // LDS bytes of the staged coefficients
    int hoist_k = 0;          // complex64: qubits of the block kept in registers
    size_t hoist_bytes = 0;   //   and its fragment bytes
    auto flush = [&]() {
        if (!cur.lop.empty()) {
            finish_pass(p, cur, dense ? S4 : S, dense);
            p.passes.push_back(cur);
        }
        cur = PassPlan();
        cur.R = R;
        cur.W = W;
        S = 0;
        S4 = 0;
        dense = false;
        staged = 0;
        hoist_k = 0;
        hoist_bytes = 0;
    };
    // Greedy packing with look-ahead: a pass opens with the first op not yet
    // placed and then scans forward, taking every op whose bits fit the tile
    // and which commutes with each op skipped so far (so it may move ahead of
    // them).  Two ops commute when neither's non-diagonal target bits meet
    // any bit of the other (shared bits are then controls or diagonal bits of
    // both).  A physical swap ends the scan.
    const size_t nl = p.lops.size();
    const size_t window = 256;
    std::vector<char> placed(nl, 0);
    // non-diagonal target bits outside the fixed bits of a register tile (6)
    // or of an LDS tile (4)
    auto need_of = [](const LOp& o, int fixed) {
        uint64_t need = 0;
        if (o.kind != LOp::DIAG)
            for (int j = 0; j < o.k; ++j)
                if (o.t[j] >= fixed) need |= 1ull << o.t[j];
        return need;
    };
    // the op joins the current pass if its bits fit (and, for complex128, its
    // staged fragments fit next to the tile)
    auto try_add = [&](size_t i) -> bool {
        const LOp& o = p.lops[i];
        const uint64_t need6 = need_of(o, 6), need4 = need_of(o, QOPS_LDS_FIXED_BITS);
        const bool d2 = dense || o.kind == LOp::DENSE || p.par.force_lds;
        const int Lt = QOPS_LDS_FIXED_BITS + cap_lds;
        const size_t sb = staged_bytes(p, o, Lt);
        const size_t tile_bytes = (size_t(1) << Lt) * (p.prec == 0 ? 8 : 16);
        size_t nstaged = staged + sb;
        int nhoist = hoist_k;
        bool lds_full;
        if (p.prec == 0) {
            // complex64: the widest 5/6-qubit matrix-core block stays in
            // registers; everything else must fit the LDS budget next to the
            // tile (two work-groups per CU)
            const bool big = o.kind == LOp::DENSE && o.k >= 5 && use_mfma_for(p, o.k, Lt);
            bool ok = true;
            if (big) {
                nstaged = staged;
                if (hoist_k == 0) {
                    nhoist = o.k;
                } else if (o.k > hoist_k) {   // the new block takes the registers
                    nhoist = o.k;
                    nstaged = staged + hoist_bytes;
                } else if (o.k == 5) {
                    nstaged = staged + sb;
                } else {
                    ok = false;               // a second 6-qubit block does not fit
                }
            }
            lds_full = !ok || nstaged + tile_bytes > lds_budget(0);
        } else {
            // complex128 passes keep all their fragments in LDS (one
            // work-group per CU)
            lds_full = d2 && staged + sb + tile_bytes > lds_budget(p.prec) && sb > 0 && staged > 0;
        }
        const int width = d2 ? __builtin_popcountll(S4 | need4) : __builtin_popcountll(S | need6);
        const int cap = d2 ? cap_lds : cap_reg;
        if (!cur.lop.empty() && (width > cap || lds_full)) return false;
        cur.lop.push_back((int)i);
        S |= need6;
        S4 |= need4;
        dense = d2;
        if (p.prec == 0 && nhoist != hoist_k) hoist_bytes = staged_bytes(p, o, Lt);
        hoist_k = nhoist;
        staged = nstaged;
        return true;
    };
    size_t first = 0;
    while (first < nl) {
        if (placed[first]) {
            ++first;
            continue;
        }
        const LOp& o0 = p.lops[first];
        if (o0.kind == LOp::PSWAP) {
            flush();
            PassPlan sp;
            sp.type = PASS_SWAP_BITS;
            sp.swap_a = o0.t[0];
            sp.swap_b = o0.t[1];
            sp.bytes_alg = state_bytes;
            sp.lop.push_back((int)first);
            p.passes.push_back(sp);
            placed[first] = 1;
            continue;
        }
        flush();
        try_add(first);
        placed[first] = 1;
        uint64_t skip_touch = 0, skip_nd = 0;
        const size_t stop = std::min(nl, first + 1 + window);
        for (size_t j = first + 1; j < stop; ++j) {
            if (placed[j]) continue;
            const LOp& o = p.lops[j];
            if (o.kind == LOp::PSWAP) break;
            const uint64_t tj = o.touch(), nj = o.tmask();
            const bool commutes = (nj & skip_touch) == 0 && (tj & skip_nd) == 0;
            if (commutes && try_add(j)) {
                placed[j] = 1;
            } else {
                skip_touch |= tj;
                skip_nd |= nj;
                if (__builtin_popcountll(skip_nd) >= n) break;   // nothing can pass any more
            }
        }
    }
    flush();
}

// Merging, fusion, packing and device-program emission of lowered
// operations (the back half of build_plan), with the plan's checks.
static Err finish_plan(Plan& p, std::vector<LOp>& lowered, std::chrono::steady_clock::time_point t0)
{
    const PlanParams& par = p.par;
    if (par.mode == QOPS_PLAN_GATEWISE) {
        p.lops.swap(lowered);
    } else {
        merge_ops(lowered, p.lops);
        if (par.merge_blocks >= 0)
            merge_dense_priced(p.lops, p.prec == QOPS_C64 ? kBlockCostC64 : kBlockCostC128);
        fuse_blocks(p.lops, std::min(par.max_fuse_k, 6));
    }
    pack(p);
    // LDS tile kernels start each of their 256 threads on a distinct tile
    // element (tiles of at least 2^8); complex64 ones read every coefficient
    // but the hoisted block's from LDS, so each such op must be staged
    for (const PassPlan& pp : p.passes)
        if (pp.type == PASS_TILE_LDS && pp.L < 8)
            return mkerr(QOPS_UNSUPPORTED, "internal: LDS tile of fewer than 2^8 amplitudes");
    if (p.prec == 0)
        for (const PassPlan& pp : p.passes) {
            if (pp.type != PASS_TILE_LDS) continue;
            const PassHdr& h = p.hdrs[pp.hdr];
            for (int i = h.op0; i < h.op0 + h.nops; ++i)
                if (i - h.op0 != h.hoist && !p.dops[i].b)
                    return mkerr(QOPS_UNSUPPORTED, "internal: an LDS-pass operation could not be staged");
            // the kernel keeps one block of 5 or 6 qubits in registers and
            // runs the others through the 5-qubit dispatch: a second block as
            // wide as 6 would be skipped there, so it must never reach it
            if (h.hoist >= 0) {
                const int hk = p.dops[h.op0 + h.hoist].a;
                if (hk != 5 && hk != 6) return mkerr(QOPS_UNSUPPORTED, "internal: hoisted block is not 5 or 6 qubits");
                for (int i = h.op0; i < h.op0 + h.nops; ++i)
                    if (i - h.op0 != h.hoist && p.dops[i].type == OP_MFMA && p.dops[i].a > 5)
                        return mkerr(QOPS_UNSUPPORTED, "internal: two 6-qubit matrix-core blocks in one LDS pass");
            }
            // the full-tile kernel runs every 5-qubit block in the 32x32x2
            // form, the smaller tiles none
            for (int i = h.op0; i < h.op0 + h.nops; ++i) {
                const DevOp& d = p.dops[i];
                const bool wide = d.type == OP_MFMA && (d.c_reg & QOPS_MFMA_WIDE) != 0;
                if (d.type == OP_MFMA && wide != (pp.L == 13 && d.a == 5))
                    return mkerr(QOPS_UNSUPPORTED, "internal: matrix-core block layout does not match the tile size");
            }
        }
    for (const PassPlan& pp : p.passes) {
        if (pp.type != PASS_TILE_LDS && pp.type != PASS_STATE_LDS) continue;
        for (int i = pp.op0; i < pp.op0 + pp.nops; ++i)
            if (p.dops[i].type == OP_MFMA && (p.dops[i].a < 3 || p.dops[i].a > 6))
                return mkerr(QOPS_UNSUPPORTED, "internal: matrix-core block outside 3..6 qubits");
    }
    p.dirty = true;
    p.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return Err{};
}


Err build_plan(int n, int prec, const int32_t* l2p_in, const qops_gate* g, size_t ng, const PlanParams& par, Plan& p)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (n < 1 || n > QOPS_MAX_QUBITS) return mkerr(QOPS_UNSUPPORTED, "n must be in [1, 34]");
    if (prec != QOPS_C64 && prec != QOPS_C128) return mkerr(QOPS_INVALID_ARG, "bad precision");
    Err e = validate_gates(n, g, ng, par.check_unitary != 0);
    if (!e.ok()) return e;
    p = Plan();
    p.n = n;
    p.prec = prec;
    p.par = par;
    if (n < 6 && p.par.mode != QOPS_PLAN_GATEWISE) p.par.state_lds_max_n = std::max(p.par.state_lds_max_n, n);
    p.l2p_in.resize(n);
    uint64_t seen = 0;
    for (int q = 0; q < n; ++q) {
        const int v = l2p_in ? l2p_in[q] : q;
        if (v < 0 || v >= n || (seen & (1ull << v))) return mkerr(QOPS_INVALID_ARG, "l2p is not a permutation");
        seen |= 1ull << v;
        p.l2p_in[q] = v;
    }
    // keep a private copy of the gate list (matrices included)
    p.gates.assign(g, g + ng);
    p.mats.resize(ng);
    for (size_t i = 0; i < ng; ++i)
        if (g[i].kind == QOPS_DENSE) {
            const size_t d = (size_t)1 << g[i].k;
            p.mats[i].assign(g[i].mat, g[i].mat + 2 * d * d);
            p.gates[i].mat = p.mats[i].data();
        } else {
            p.gates[i].mat = nullptr;
        }
    std::vector<int> l2p = p.l2p_in;
    std::vector<LOp> lowered;
    if (par.remap && n > 6 && par.mode != QOPS_PLAN_GATEWISE) {
        // Profile-guided remap (virtual swap, paper Sec. III-D): the qubits
        // that non-diagonal gates target most often are moved into physical
        // bits 0..5, which every tile pass holds, by bit exchanges up front.
        std::vector<long> hits(n, 0);
        for (size_t i = 0; i < ng; ++i) {
            const qops_gate& g = p.gates[i];
            if (diag_kind(g.kind) || g.kind == QOPS_SWAP) continue;
            const int k = g.kind == QOPS_DENSE ? g.k : gate_arity(g.kind);
            if (g.kind == QOPS_CX) hits[g.q[1]]++;
            else
                for (int j = 0; j < k; ++j) hits[g.q[j]]++;
        }
        std::vector<int> order(n);
        for (int q = 0; q < n; ++q) order[q] = q;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hits[a] > hits[b]; });
        std::vector<bool> hot(n, false);
        for (int i = 0; i < 6; ++i) hot[order[i]] = hits[order[i]] > 0;
        std::vector<int> p2l(n);
        for (int q = 0; q < n; ++q) p2l[l2p[q]] = q;
        for (int i = 0; i < 6; ++i) {
            const int q = order[i];
            if (!hot[q] || l2p[q] < 6) continue;
            int slot = -1;
            for (int b = 0; b < 6 && slot < 0; ++b)
                if (!hot[p2l[b]]) slot = b;
            if (slot < 0) break;
            LOp o;
            o.kind = LOp::PSWAP;
            o.k = 2;
            o.t[0] = slot;
            o.t[1] = l2p[q];
            lowered.push_back(o);
            const int other = p2l[slot];
            std::swap(l2p[q], l2p[other]);
            p2l[l2p[q]] = q;
            p2l[l2p[other]] = other;
        }
    }
    // rotation folding (paper Sec. III-D): on request, or by the paper's rule
    // (T gates above 10% of the circuit) unless switched off
    const qops_gate* lg = p.gates.data();
    size_t lng = ng;
    std::vector<qops_gate> folded;
    p.n_folded = 0;
    if (par.mode != QOPS_PLAN_GATEWISE &&
        (par.fold > 0 || (par.fold == 0 && fold_rule_fires(p.gates.data(), ng)))) {
        fold_rotations(n, p.gates.data(), ng, folded, p.n_folded);
        lg = folded.data();
        lng = folded.size();
    }
    e = lower(n, lg, lng, par.swap_mode, l2p, lowered, p.n_virtual_swaps);
    if (!e.ok()) return e;
    p.l2p_out = l2p;
    return finish_plan(p, lowered, t0);
}

Err plan_from_lops(int n, int prec, std::vector<LOp>& ops, const PlanParams& par, Plan& p)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (n < 1 || n > QOPS_MAX_QUBITS) return mkerr(QOPS_UNSUPPORTED, "n must be in [1, 34]");
    p = Plan();
    p.n = n;
    p.prec = prec;
    p.par = par;
    if (n < 6 && p.par.mode != QOPS_PLAN_GATEWISE) p.par.state_lds_max_n = std::max(p.par.state_lds_max_n, n);
    p.l2p_in.resize(n);
    for (int q = 0; q < n; ++q) p.l2p_in[q] = q;
    p.l2p_out = p.l2p_in;
    for (const LOp& o : ops) {
        const uint64_t bad = n >= 64 ? 0 : ~((1ull << n) - 1);
        if (o.touch() & bad) return mkerr(QOPS_QUBIT_RANGE, "internal: lowered op outside the state");
    }
    return finish_plan(p, ops, t0);
}

Err lower_gates(int n, const qops_gate* g, size_t ng, int swap_mode, std::vector<int>& l2p, std::vector<LOp>& out,
                int& nvirt)
{
    Err e = validate_gates(n, g, ng, false);
    if (!e.ok()) return e;
    return lower(n, g, ng, swap_mode, l2p, out, nvirt);
}

Err update_plan(Plan& p, const qops_gate* g, size_t ng)
{
    if (ng != p.gates.size()) return mkerr(QOPS_BAD_STATE, "gate count differs from the plan");
    for (size_t i = 0; i < ng; ++i) {
        const qops_gate& a = p.gates[i];
        const qops_gate& b = g[i];
        if (a.kind != b.kind || a.k != b.k || a.n_ctrl != b.n_ctrl)
            return mkerr(QOPS_BAD_STATE, "gate structure differs from the plan");
        const int k = a.kind == QOPS_DENSE ? a.k : gate_arity(a.kind);
        for (int j = 0; j < k; ++j)
            if (a.q[j] != b.q[j]) return mkerr(QOPS_BAD_STATE, "gate qubits differ from the plan");
        for (int j = 0; j < a.n_ctrl; ++j)
            if (a.ctrl[j] != b.ctrl[j]) return mkerr(QOPS_BAD_STATE, "gate controls differ from the plan");
    }
    // Re-plan with identical structure: merging decisions depend only on the
    // structure, except identity cancellation, which is re-evaluated.
    Plan q;
    Err e = build_plan(p.n, p.prec, p.l2p_in.data(), g, ng, p.par, q);
    if (!e.ok()) return e;
    std::swap(q.d_hdr, p.d_hdr);
    std::swap(q.d_ops, p.d_ops);
    std::swap(q.d_coef, p.d_coef);
    q.predicted_s = p.predicted_s;
    p = std::move(q);
    p.dirty = true;
    return Err{};
}

void pass_features(const Plan& p, const PassPlan& pp, float* f)
{
    for (int i = 0; i < kNumFeatures; ++i) f[i] = 0.f;
    f[0] = p.n / 32.f;
    f[1] = (float)p.prec;
    f[2 + (int)pp.type] = 1.f;
    f[7] = pp.L / 16.f;
    f[8] = pp.n_lane_ops / 16.f;
    f[9] = pp.n_reg_ops / 16.f;
    f[10] = pp.n_diag_ops / 16.f;
    f[11] = pp.n_remaps / 4.f;
    f[12] = pp.n_dense / 8.f;
    f[13] = pp.n_mfma / 8.f;
    f[14] = pp.max_k / 6.f;
    f[15] = (float)(pp.flops / (8.0 * std::ldexp(1.0, p.n) * 64.0));
    f[16] = (float)pp.W;
    f[17] = (float)pp.R / 5.f;
    uint64_t touched = 0;
    int nctrl = 0, ksum = 0, nk = 0;
    for (int li : pp.lop) {
        const LOp& o = p.lops[li];
        touched |= o.touch();
        if (o.kind == LOp::DIAG) {
            for (int j = 0; j < o.k; ++j) touched |= 1ull << o.t[j];
        }
        if (o.cmask) ++nctrl;
        ksum += o.k;
        ++nk;
        if (o.kind == LOp::DENSE && o.k >= 1 && o.k <= 6) f[55 + o.k - 1] += 1.f / 8.f;
    }
    for (int b = 0; b < 32 && b < 64; ++b)
        if (touched & (1ull << b)) f[18 + b] = 1.f;
    int lo = -1, hi = -1;
    for (int b = 6; b < 64; ++b)
        if (touched & (1ull << b)) {
            if (lo < 0) lo = b;
            hi = b;
        }
    f[50] = lo < 0 ? 0.f : lo / 32.f;
    f[51] = hi < 0 ? 0.f : hi / 32.f;
    f[52] = nctrl / 16.f;
    f[53] = nk ? (float)ksum / nk / 6.f : 0.f;
    f[54] = (float)pp.nops / 64.f;
    f[61] = (float)(pp.bytes_alg / (16.0 * std::ldexp(1.0, p.n)));
    f[62] = pp.type == PASS_SWAP_BITS ? 1.f : 0.f;
    f[63] = 1.f;   // bias-like constant
}

}  // namespace qops
