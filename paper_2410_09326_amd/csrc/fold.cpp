// Rotation folding (paper Sec. III-D): diagonal phases that act on the same
// parity of the circuit's path variables are merged into one, across CNOT,
// X and SWAP gates and across unrelated gates.
//
// Every wire carries an affine parity of path variables: a wire starts as its
// own variable; X flips the constant; CNOT adds the control's parity to the
// target's; SWAP exchanges parities; diagonal gates keep every parity; any
// other gate gives its targets fresh variables.  A one-qubit phase gate (RZ,
// P, S, T, Z and their inverses) multiplies each path by exp(i theta f) for
// the parity f its wire carries, a scalar per path, so two such phases on the
// same parity add no matter where they sit.  The first occurrence of each
// parity keeps its position (a P gate on its wire) and collects the angles of
// the later ones; constant parities and the RZ offsets become one global
// phase, emitted at the end as P(2a) RZ(-2a) on qubit 0, so the folded
// circuit equals the input exactly (not just up to a phase).  Two-qubit
// diagonals (CZ, CP, RZZ) are kept as gates: split into parity phases they
// would cost more operations than the folding saves.
#include <cmath>
#include <map>
#include <vector>

#include "planner.hpp"

namespace qops {
namespace {

struct Parity {
    std::vector<uint64_t> w;   // variable bitset
    bool c = false;            // affine constant
};

void xor_into(Parity& a, const Parity& b)
{
    if (a.w.size() < b.w.size()) a.w.resize(b.w.size(), 0);
    for (size_t i = 0; i < b.w.size(); ++i) a.w[i] ^= b.w[i];
    a.c ^= b.c;
}

std::vector<uint64_t> key_of(const Parity& a)
{
    std::vector<uint64_t> k = a.w;
    while (!k.empty() && k.back() == 0) k.pop_back();
    return k;
}

qops_gate make_gate(int kind, int a, int b, double theta)
{
    qops_gate g{};
    g.kind = (uint16_t)kind;
    g.k = (uint8_t)(b >= 0 ? 2 : 1);
    g.n_ctrl = 0;
    g.q[0] = a;
    if (b >= 0) g.q[1] = b;
    g.param[0] = theta;
    g.mat = nullptr;
    return g;
}

}  // namespace

bool fold_rule_fires(const qops_gate* g, size_t ng)
{
    // the activation rule of the paper: T gates above 10% of all gates
    size_t t = 0;
    for (size_t i = 0; i < ng; ++i) t += (g[i].kind == QOPS_T || g[i].kind == QOPS_TDG) ? 1 : 0;
    return ng > 0 && 10 * t > ng;
}

void fold_rotations(int n, const qops_gate* in, size_t ng, std::vector<qops_gate>& out, int& removed)
{
    struct Term {
        size_t pos;     // index of its placeholder in `out`
        int a;          // wire carrying the parity at its first occurrence
        bool wc;        // constant of those wires' parity
        double theta;   // collected angle of exp(i theta v), v the variable part
    };
    std::vector<Parity> lab((size_t)n);
    int nv = 0;
    auto fresh = [&](int q) {
        Parity p;
        p.w.assign((size_t)nv / 64 + 1, 0);
        p.w[(size_t)nv / 64] |= 1ull << (nv % 64);
        ++nv;
        lab[(size_t)q] = p;
    };
    for (int q = 0; q < n; ++q) fresh(q);
    std::map<std::vector<uint64_t>, size_t> first;
    std::vector<Term> terms;
    double gphase = 0.0;
    int phase_in = 0;
    out.clear();
    out.reserve(ng + 2);
    // phase exp(i theta f) on the parity f (with its constant) that wire a
    // carries now
    auto add_term = [&](const Parity& f, double theta, int a) {
        double th = theta;
        if (f.c) {   // exp(i t (v xor 1)) = exp(i t) exp(-i t v)
            gphase += theta;
            th = -theta;
        }
        const std::vector<uint64_t> k = key_of(f);
        if (k.empty()) return;   // constant parity: already in gphase
        auto it = first.find(k);
        if (it != first.end()) {
            terms[it->second].theta += th;
            return;
        }
        Term t;
        t.pos = out.size();
        t.a = a;
        t.wc = f.c;
        t.theta = th;
        first.emplace(k, terms.size());
        terms.push_back(t);
        out.push_back(qops_gate{});   // placeholder
    };
    for (size_t i = 0; i < ng; ++i) {
        const qops_gate& g = in[i];
        const int a = g.q[0], b = g.q[1];
        if (g.n_ctrl > 0) {
            // controlled forms: diagonal ones keep every parity, others give
            // their targets fresh variables
            out.push_back(g);
            if (!diag_kind(g.kind)) {
                const int k = g.kind == QOPS_DENSE ? g.k : gate_arity(g.kind);
                if (g.kind == QOPS_CX) fresh(b);
                else
                    for (int j = 0; j < k; ++j) fresh(g.q[j]);
            }
            continue;
        }
        switch (g.kind) {
        case QOPS_X:
            out.push_back(g);
            lab[(size_t)a].c = !lab[(size_t)a].c;
            break;
        case QOPS_CX:
            out.push_back(g);
            xor_into(lab[(size_t)b], lab[(size_t)a]);
            break;
        case QOPS_SWAP:
            out.push_back(g);
            std::swap(lab[(size_t)a], lab[(size_t)b]);
            break;
        case QOPS_Z: ++phase_in; add_term(lab[(size_t)a], M_PI, a); break;
        case QOPS_S: ++phase_in; add_term(lab[(size_t)a], M_PI / 2, a); break;
        case QOPS_SDG: ++phase_in; add_term(lab[(size_t)a], -M_PI / 2, a); break;
        case QOPS_T: ++phase_in; add_term(lab[(size_t)a], M_PI / 4, a); break;
        case QOPS_TDG: ++phase_in; add_term(lab[(size_t)a], -M_PI / 4, a); break;
        case QOPS_P: ++phase_in; add_term(lab[(size_t)a], g.param[0], a); break;
        case QOPS_RZ:   // diag(e^{-it/2}, e^{it/2}) = e^{-it/2} e^{i t x}
            ++phase_in;
            gphase -= g.param[0] / 2;
            add_term(lab[(size_t)a], g.param[0], a);
            break;
        case QOPS_CZ:
        case QOPS_CP:
        case QOPS_RZZ:
            // two-qubit diagonals stay as they are (they keep every parity)
            out.push_back(g);
            break;
        default: {   // non-diagonal: fresh variables on every target
            out.push_back(g);
            const int k = g.kind == QOPS_DENSE ? g.k : gate_arity(g.kind);
            for (int j = 0; j < k; ++j) fresh(g.q[j]);
            break;
        }
        }
    }
    // emit every collected term at its first position
    std::vector<char> keep(out.size(), 1);
    int emitted = 0;
    for (const Term& t : terms) {
        double phi = t.theta;
        if (t.wc) {   // the wires carry v xor 1: exp(i phi v) = e^{i phi} exp(-i phi p)
            gphase += phi;
            phi = -phi;
        }
        if (phi == 0.0) {
            keep[t.pos] = 0;
            continue;
        }
        out[t.pos] = make_gate(QOPS_P, t.a, -1, phi);
        ++emitted;
    }
    std::vector<qops_gate> res;
    res.reserve(out.size() + 2);
    for (size_t i = 0; i < out.size(); ++i)
        if (keep[i]) res.push_back(out[i]);
    const double gp = std::remainder(gphase, 2.0 * M_PI);
    if (gp != 0.0 && n > 0) {   // e^{i a} = P(2a) RZ(-2a) on any qubit
        res.push_back(make_gate(QOPS_P, 0, -1, 2.0 * gp));
        res.push_back(make_gate(QOPS_RZ, 0, -1, -2.0 * gp));
        emitted += 2;
    }
    out.swap(res);
    removed = phase_in - emitted;
}

}  // namespace qops
