// State-vector kernels for gfx950 (CDNA4, wave64).
//
// Tile pass (the "chunk segment" of the paper's storage simulator, Sec. II-B,
// mapped onto the GPU memory hierarchy): a work-group owns a tile of 2^L
// amplitudes.  Tile positions 0..5 are physical bits 0..5 and are held one
// per lane, so every load/store of a wave is 64 consecutive amplitudes;
// gates on those bits use cross-lane shuffles.  The upper positions are split
// into R register bits (gates applied in registers) and W wave bits (changed
// by a remap through LDS).  Dense k-qubit blocks run on the LDS copy of the
// tile, on the vector ALU or on matrix cores (MFMA, 16x16x4 f32 / f64).
// One read and one write of the state per pass, however many gates it holds.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "devprog.hpp"
#include "kernels.hpp"

namespace qops {

// Compile-time loop: calls f(std::integral_constant<int, I>) for I = 0..N-1,
// so that every register index is a constant and the state stays in VGPRs.
template <int I, int N, typename F>
__device__ __forceinline__ void sfor_impl(F& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        sfor_impl<I + 1, N>(f);
    }
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f)
{
    sfor_impl<0, N>(f);
}

template <typename T> struct CxT;
template <> struct CxT<float> { using V = float2; using A4 = float __attribute__((ext_vector_type(4))); };
template <> struct CxT<double> { using V = double2; using A4 = double __attribute__((ext_vector_type(4))); };

template <typename V>
__device__ __forceinline__ V cmul(V a, V b)
{
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// m0*x0 + m1*x1 (complex)
template <typename V>
__device__ __forceinline__ V cdot2(V m0, V x0, V m1, V x1)
{
    V r;
    r.x = m0.x * x0.x - m0.y * x0.y + m1.x * x1.x - m1.y * x1.y;
    r.y = m0.x * x0.y + m0.y * x0.x + m1.x * x1.y + m1.y * x1.x;
    return r;
}

// Component-wise select by value (a conditional on two struct lvalues would
// select an address and pin the register array in scratch memory).
template <typename V>
__device__ __forceinline__ V csel(bool c, V a, V b)
{
    V r;
    r.x = c ? a.x : b.x;
    r.y = c ? a.y : b.y;
    return r;
}

template <typename T>
__device__ __forceinline__ typename CxT<T>::V ldc(const T* __restrict__ c, int i)
{
    typename CxT<T>::V v;
    v.x = c[2 * i];
    v.y = c[2 * i + 1];
    return v;
}

// LDS slot of tile element e: the low five bits (32 amplitudes = one row of
// the 64 four-byte banks for complex64) are XORed with the next five, so
// that strided groups and matrix-core column sets spread over the banks.
// A bijection on [0, 2^L) for every L >= 5.
// GF(2)-linear: swz(a ^ b) = swz(a) ^ swz(b).
__host__ __device__ constexpr uint32_t swz(uint32_t e) { return e ^ ((e >> 5) & 31u); }

// Inserts a zero bit at every set position of `mask` (ascending) into g.
__device__ __forceinline__ uint32_t spread_mask(uint32_t g, uint32_t mask)
{
    while (mask) {
        const int p = __builtin_ctz(mask);
        mask &= mask - 1;
        const uint32_t low = g & ((1u << p) - 1u);
        g = ((g >> p) << (p + 1)) | low;
    }
    return g;
}

// Bits of g, lowest first, placed at the set positions of dmask (lowest first).
__device__ __forceinline__ uint32_t deposit_bits(uint32_t g, uint32_t dmask)
{
    uint32_t r = 0;
    while (dmask) {
        const uint32_t low = dmask & (0u - dmask);
        if (g & 1u) r |= low;
        g >>= 1;
        dmask &= dmask - 1u;
    }
    return r;
}

__device__ __forceinline__ uint64_t spread_mask64(uint64_t g, uint64_t mask)
{
    while (mask) {
        const int p = __builtin_ctzll(mask);
        mask &= mask - 1;
        const uint64_t low = g & ((1ull << p) - 1ull);
        g = ((g >> p) << (p + 1)) | low;
    }
    return g;
}

// ---------------------------------------------------------------------------
// Register-resident operations
// ---------------------------------------------------------------------------

// 2x2 on register bit B.  Register-slot controls `creg` are compile-time per
// slot and uniform; `tok` is the per-lane control result.
// Exact X on register bit B: exchange the two halves (no arithmetic).
template <int B, int R, bool CTRL, typename V>
__device__ __forceinline__ void xgate_reg_b(V (&a)[1 << R], uint32_t creg, bool tok)
{
    sfor<(1 << R)>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (!(j & (1 << B))) {
            constexpr int j1 = j | (1 << B);
            if (!CTRL || ((uint32_t)j & creg) == creg) {
                const V x0 = a[j], x1 = a[j1];
                if (CTRL) {
                    a[j] = csel(tok, x1, x0);
                    a[j1] = csel(tok, x0, x1);
                } else {
                    a[j] = x1;
                    a[j1] = x0;
                }
            }
        }
    });
}

template <int R, bool CTRL, typename V>
__device__ __forceinline__ void xgate_reg(int b, V (&a)[1 << R], uint32_t creg, bool tok)
{
    switch (b) {
    case 0: xgate_reg_b<0, R, CTRL>(a, creg, tok); break;
    case 1: if constexpr (R > 1) xgate_reg_b<1, R, CTRL>(a, creg, tok); break;
    case 2: if constexpr (R > 2) xgate_reg_b<2, R, CTRL>(a, creg, tok); break;
    case 3: if constexpr (R > 3) xgate_reg_b<3, R, CTRL>(a, creg, tok); break;
    case 4: if constexpr (R > 4) xgate_reg_b<4, R, CTRL>(a, creg, tok); break;
    case 5: if constexpr (R > 5) xgate_reg_b<5, R, CTRL>(a, creg, tok); break;
    default: break;
    }
}

template <int B, int R, bool CTRL, typename V>
__device__ __forceinline__ void oneq_reg_b(V (&a)[1 << R], V m00, V m01, V m10, V m11, uint32_t creg, bool tok)
{
    sfor<(1 << R)>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (!(j & (1 << B))) {
            constexpr int j1 = j | (1 << B);
            if (!CTRL || ((uint32_t)j & creg) == creg) {
                const V x0 = a[j], x1 = a[j1];
                const V y0 = cdot2(m00, x0, m01, x1);
                const V y1 = cdot2(m10, x0, m11, x1);
                if (CTRL) {
                    a[j] = csel(tok, y0, x0);
                    a[j1] = csel(tok, y1, x1);
                } else {
                    a[j] = y0;
                    a[j1] = y1;
                }
            }
        }
    });
}

template <int R, bool CTRL, typename V>
__device__ __forceinline__ void oneq_reg(int b, V (&a)[1 << R], V m00, V m01, V m10, V m11, uint32_t creg, bool tok)
{
    switch (b) {
    case 0: oneq_reg_b<0, R, CTRL>(a, m00, m01, m10, m11, creg, tok); break;
    case 1: if constexpr (R > 1) oneq_reg_b<1, R, CTRL>(a, m00, m01, m10, m11, creg, tok); break;
    case 2: if constexpr (R > 2) oneq_reg_b<2, R, CTRL>(a, m00, m01, m10, m11, creg, tok); break;
    case 3: if constexpr (R > 3) oneq_reg_b<3, R, CTRL>(a, m00, m01, m10, m11, creg, tok); break;
    case 4: if constexpr (R > 4) oneq_reg_b<4, R, CTRL>(a, m00, m01, m10, m11, creg, tok); break;
    case 5: if constexpr (R > 5) oneq_reg_b<5, R, CTRL>(a, m00, m01, m10, m11, creg, tok); break;
    default: break;
    }
}

// Cross-lane exchange through ds_bpermute; `addr` = 4 * (lane ^ mask).
__device__ __forceinline__ float shfl_xor_f(float v, int addr)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double shfl_xor_f(double v, int addr)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Exact X on lane bit t: take the partner's amplitude.
template <int R, bool CTRL, typename V>
__device__ __forceinline__ void xgate_lane(int t, int lane, V (&a)[1 << R], uint32_t creg, bool tok)
{
    const int addr = (lane ^ (1 << t)) << 2;
    sfor<(1 << R)>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (!CTRL || ((uint32_t)j & creg) == creg) {
            V p;
            p.x = shfl_xor_f(a[j].x, addr);
            p.y = shfl_xor_f(a[j].y, addr);
            a[j] = CTRL ? csel(tok, p, a[j]) : p;
        }
    });
}

// 2x2 on lane bit t: each lane computes its own output from its amplitude
// and its partner's (lane ^ 2^t).
template <int R, bool CTRL, typename V>
__device__ __forceinline__ void oneq_lane(int t, int lane, V (&a)[1 << R], V m00, V m01, V m10, V m11,
                                          uint32_t creg, bool tok)
{
    const bool hi = (lane >> t) & 1;
    const V ms = csel(hi, m11, m00);
    const V mo = csel(hi, m10, m01);
    const int addr = (lane ^ (1 << t)) << 2;
    sfor<(1 << R)>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (!CTRL || ((uint32_t)j & creg) == creg) {
            V p;
            p.x = shfl_xor_f(a[j].x, addr);
            p.y = shfl_xor_f(a[j].y, addr);
            const V y = cdot2(ms, a[j], mo, p);
            if (CTRL)
                a[j] = csel(tok, y, a[j]);
            else
                a[j] = y;
        }
    });
}

// ---------------------------------------------------------------------------
// LDS-resident operations (tile of 2^L amplitudes at `lds`)
// ---------------------------------------------------------------------------

// Fused multiply-add in the state precision.
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Dense 2^K x 2^K on tile positions pos[0..K-1] (matrix bit order), vector
// ALU.  Every thread handles whole groups.  Group g of the tile has its
// target bits zero and its other bits taken from g in order; the insertion
// is GF(2)-linear, as is the LDS swizzle, so the byte offsets of a thread's
// groups are one XOR of a per-thread part and a per-iteration part.  The
// coefficients are read once per operation; each complex product-sum is
// four fused multiply-adds.
template <int K, typename T>
__device__ void dense_lds(typename CxT<T>::V* lds, int L, const DevOp& op, const T* __restrict__ U, int tid,
                          int nthr)
{
    using V = typename CxT<T>::V;
    constexpr int D = 1 << K;
    uint32_t mask = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) mask |= 1u << op.pos[j];
    uint32_t toff[D];
#pragma unroll
    for (int s = 0; s < D; ++s) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (s & (1 << j)) o |= 1u << op.pos[j];
        toff[s] = swz(o) * (uint32_t)sizeof(V);
    }
    T ur[D * D], ui[D * D];
    if constexpr (K <= 2) {
#pragma unroll
        for (int i = 0; i < D * D; ++i) {
            ur[i] = U[2 * i];
            ui[i] = U[2 * i + 1];
        }
    }
    const uint32_t ngroups = 1u << (L - K);
    const uint32_t gt = spread_mask((uint32_t)tid, mask);   // tid < nthr <= ngroups or no group at all
    const uint32_t tsw = swz(gt) * (uint32_t)sizeof(V);
    unsigned char* base = reinterpret_cast<unsigned char*>(lds);
    for (uint32_t g0 = 0; g0 + (uint32_t)tid < ngroups; g0 += (uint32_t)nthr) {
        const uint32_t gu = spread_mask(g0, mask);          // uniform part
        const uint32_t gb = gt ^ gu;
        if ((gb & op.c_tile) != op.c_tile) continue;
        const uint32_t off = tsw ^ (swz(gu) * (uint32_t)sizeof(V));
        V in[D];
#pragma unroll
        for (int s = 0; s < D; ++s) in[s] = *reinterpret_cast<const V*>(base + (off ^ toff[s]));
#pragma unroll
        for (int r = 0; r < D; ++r) {
            T ax, ay;
            if constexpr (K <= 2) {
                ax = ur[r * D] * in[0].x;
                ay = ur[r * D] * in[0].y;
                ax = fmat(-ui[r * D], in[0].y, ax);
                ay = fmat(ui[r * D], in[0].x, ay);
#pragma unroll
                for (int c = 1; c < D; ++c) {
                    ax = fmat(ur[r * D + c], in[c].x, ax);
                    ax = fmat(-ui[r * D + c], in[c].y, ax);
                    ay = fmat(ur[r * D + c], in[c].y, ay);
                    ay = fmat(ui[r * D + c], in[c].x, ay);
                }
            } else {
                ax = 0;
                ay = 0;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const T cr = U[2 * (r * D + c)], ci = U[2 * (r * D + c) + 1];
                    ax = fmat(cr, in[c].x, ax);
                    ax = fmat(-ci, in[c].y, ax);
                    ay = fmat(cr, in[c].y, ay);
                    ay = fmat(ci, in[c].x, ay);
                }
            }
            V w;
            w.x = ax;
            w.y = ay;
            *reinterpret_cast<V*>(base + (off ^ toff[r])) = w;
        }
    }
}

template <typename T>
__device__ void dense_lds_dispatch(typename CxT<T>::V* lds, int L, const DevOp& op, const T* __restrict__ U,
                                   int tid, int nthr)
{
    switch (op.a) {
    case 1: dense_lds<1, T>(lds, L, op, U, tid, nthr); break;
    case 2: dense_lds<2, T>(lds, L, op, U, tid, nthr); break;
    case 3: dense_lds<3, T>(lds, L, op, U, tid, nthr); break;
    case 4: if constexpr (sizeof(T) == 4) dense_lds<4, T>(lds, L, op, U, tid, nthr); break;
    default: break;
    }
}

// Diagonal table over m = op.a bits, in LDS.  Bit i of the table index is
// tile position v (pos[i] = enc_src(SRC_LANE, v)) or physical bit v of the
// tile's base index (pos[i] = enc_src(SRC_GLOB, v)).
template <typename T>
__device__ void diag_lds(typename CxT<T>::V* lds, int L, const DevOp& op, const T* __restrict__ tab, uint64_t base,
                         int tid, int nthr)
{
    const int m = op.a;
    uint32_t iglob = 0, tmask[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        tmask[i] = 0;
        if (i < m) {
            const int cls = op.pos[i] >> 8, v = op.pos[i] & 255;
            if (cls == SRC_GLOB) iglob |= (uint32_t)((base >> v) & 1ull) << i;
            else tmask[i] = 1u << v;
        }
    }
    const uint32_t N = 1u << L;
    for (uint32_t x = tid; x < N; x += nthr) {
        uint32_t idx = iglob;
#pragma unroll
        for (int i = 0; i < 6; ++i)
            if (x & tmask[i]) idx |= 1u << i;
        lds[swz(x)] = cmul(lds[swz(x)], ldc(tab, (int)idx));
    }
}

// Dense 2^K x 2^K on tile positions with matrix cores (four waves).  The block
// is the real embedding M (2^(K+1) square, rows/cols interleaved re,im)
// applied to the tile viewed as a 2^(K+1) x 2^(L-K) real matrix (one column
// per group of 2^K amplitudes, 16 columns per column block).  The waves form
// RW row groups x CW column groups.  A wave keeps the A fragments of all its
// row blocks in registers for the whole operation and feeds every B value it
// reads to all of them.  With RW = 1 every column block belongs to one wave,
// which reads, multiplies and writes it back without synchronisation; with
// RW > 1 the waves of a column group finish reading a chunk of column blocks
// before any of them writes it (one barrier per chunk).
// A fragments are pre-arranged by the host (rows permuted for f64 so both
// precisions return the same D layout): lane l, register i of the result
// holds real row 4(l/16)+i of column l%16; the B operand of lane l is real
// row 4 ks + l/16 of column l%16.  LDS slots are swizzled (swz), whose
// linearity turns every address into one XOR of a per-lane and a uniform part.
// LDS element access by byte offset (the XOR-swizzled addresses of the
// matrix-core loops are formed on byte offsets, one XOR per access).
template <typename V>
__device__ __forceinline__ V lds_at(const V* lds, uint32_t off)
{
    return *reinterpret_cast<const V*>(reinterpret_cast<const unsigned char*>(lds) + off);
}
template <typename V>
__device__ __forceinline__ void lds_put(V* lds, uint32_t off, const V& v)
{
    *reinterpret_cast<V*>(reinterpret_cast<unsigned char*>(lds) + off) = v;
}

template <int K, typename T>
struct MfmaShape {
    // K = 3: the real embedding (2^(K+1) real rows, re/im interleaved).
    // K >= 4: Gauss's three-product form on complex rows: with U = A + iB
    // and a column x + iy, T1 = A x, T2 = B y, T3 = (A + B)(x + y) give
    // Re = T1 - T2 and Im = T3 - T1 - T2 (3/4 of the real embedding's MFMAs)
    static constexpr bool G = K >= 4;
    static constexpr int KS = G ? 1 << (K - 2) : 1 << (K - 1);   // k-steps of 4 rows
    static constexpr int RB = G ? 1 << (K - 4) : 1 << (K - 3);   // row blocks of 16 rows
    static constexpr int RW = G ? RB : 1;                        // waves per column group
    static constexpr int CW = 4 / RW;                            // column groups
    static constexpr int RPW = RB / RW;                          // row blocks per wave
    static constexpr int NF = G ? 3 : RPW;                       // fragment sets per wave
    // column blocks in flight (one barrier per chunk if RW > 1)
    static constexpr int CH = 4;
};

// The A fragments of a wave's row blocks (registers).
template <int K, typename T>
using MfmaFrag = T[MfmaShape<K, T>::NF][MfmaShape<K, T>::KS];

// The A fragments of the wave's row blocks, from global memory or LDS
// (Gauss form: A, B and A + B of the wave's row block, per k-step).
template <int K, typename T>
__device__ __forceinline__ void mfma_load_a(MfmaFrag<K, T>& av, const T* __restrict__ A, int lane, int wave)
{
    using S = MfmaShape<K, T>;
    const int rg = wave % S::RW;
    if constexpr (S::G) {
#pragma unroll
        for (int ks = 0; ks < S::KS; ++ks)
#pragma unroll
            for (int m = 0; m < 3; ++m) av[m][ks] = A[((rg * S::KS + ks) * 3 + m) * 64 + lane];
    } else {
#pragma unroll
        for (int r = 0; r < S::RPW; ++r)
#pragma unroll
            for (int ks = 0; ks < S::KS; ++ks) av[r][ks] = A[((rg * S::RPW + r) * S::KS + ks) * 64 + lane];
    }
}

// Gauss form of a 2^K x 2^K complex block (K >= 4): wave (rb, cg) computes
// complex rows 16 rb .. 16 rb + 15 of its columns.  The B operand of lane l
// in k-step ks is input 4 ks + l/16 of column l%16, read as one (re, im)
// pair; the result rows 4(l/16) + i, i < 4, of column l%16 come back in
// registers i of the three accumulators.
template <int K, typename T>
__device__ __forceinline__ void mfma_core_gauss(typename CxT<T>::V* lds, int L, const DevOp& op,
                                                const MfmaFrag<K, T>& av, int lane, int wave)
{
    using V = typename CxT<T>::V;
    using A4 = typename CxT<T>::A4;
    using S = MfmaShape<K, T>;
    constexpr int KS = S::KS, RW = S::RW, CW = S::CW, CH = S::CH;
    const int rb = wave % RW, cg = wave / RW;
    const int ncb = 1 << (L - K - 4);
    const int nper = (ncb + CW - 1) / CW;      // same for every wave
    uint32_t bit[K];
#pragma unroll
    for (int j = 0; j < K; ++j) bit[j] = 1u << op.pos[j];
    const uint32_t gl = deposit_bits((uint32_t)(lane & 15), op.c_lane);
    auto toff = [&](uint32_t s) {              // s is a compile-time constant or lane-uniform
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (s & (1u << j)) o |= bit[j];
        return o;
    };
    const uint32_t krow = (uint32_t)(lane >> 4);
    const uint32_t in_sw = swz(toff(krow));                 // input bits 0, 1
    const uint32_t out_sw = swz(toff(4u * krow)) ^ swz(toff(16u * (uint32_t)rb));
    const uint32_t wmask = op.c_wave;
    const uint32_t wstep = deposit_bits((uint32_t)CW, wmask);
    uint32_t gblk = deposit_bits((uint32_t)cg, wmask);
    auto mfma = [](const T a, const T b, const A4 c) -> A4 {
        if constexpr (sizeof(T) == 4) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
        else return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    };
    // issue priority over the other work-group's waves on this SIMD while
    // the wave streams MFMAs and writes their results back (the other
    // work-group's tile loads and stores fill the matrix core's gaps instead
    // of delaying it)
    __builtin_amdgcn_s_setprio(1);
    for (int i0 = 0; i0 < nper; i0 += CH) {
        A4 d1[CH], d2[CH], d3[CH];
        uint32_t gsw[CH], gcol[CH], gin[CH];
        bool ok[CH];
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            const int blk = cg + (i0 + c) * CW;
            ok[c] = i0 + c < nper && blk < ncb;
            d1[c] = A4{0, 0, 0, 0};
            d2[c] = A4{0, 0, 0, 0};
            d3[c] = A4{0, 0, 0, 0};
            gcol[c] = gl | gblk;
            gsw[c] = swz(gcol[c]);
            gin[c] = (gsw[c] ^ in_sw) * (uint32_t)sizeof(V);   // byte offsets: one XOR per access
            gblk = ((gblk | ~wmask) + wstep) & wmask;
        });
        // B values (and x + y) one k-step ahead of the MFMAs that use them:
        // the sums of step ks + 1 are formed while the MFMAs of step ks run,
        // so no MFMA waits on the vector ALU result it reads
        V bq[2][CH];
        T bs[2][CH];
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            bq[0][c] = lds_at(lds, gin[c]);
        });
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            bs[0][c] = bq[0][c].x + bq[0][c].y;
        });
        sfor<KS>([&](auto kc) {
            constexpr int ks = decltype(kc)::value;
            constexpr int cur = ks & 1;
            if constexpr (ks + 1 < KS) {
                const uint32_t nx = swz(toff((uint32_t)(4 * (ks + 1)))) * (uint32_t)sizeof(V);
                sfor<CH>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    bq[cur ^ 1][c] = lds_at(lds, gin[c] ^ nx);
                });
            }
            __builtin_amdgcn_sched_barrier(0);
            sfor<CH>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
                d1[c] = mfma(av[0][ks], bq[cur][c].x, d1[c]);
                d2[c] = mfma(av[1][ks], bq[cur][c].y, d2[c]);
                d3[c] = mfma(av[2][ks], bs[cur][c], d3[c]);
            });
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (ks + 1 < KS) {
                sfor<CH>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    bs[cur ^ 1][c] = bq[cur ^ 1][c].x + bq[cur ^ 1][c].y;
                });
                __builtin_amdgcn_sched_barrier(0);
            }
        });
        if constexpr (RW > 1) __syncthreads();   // the chunk's inputs are read
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            if (ok[c] && (gcol[c] & op.c_tile) == op.c_tile) {
                uint32_t g_out = (gsw[c] ^ out_sw) * (uint32_t)sizeof(V);
                asm volatile("" : "+v"(g_out));   // keeps the byte form (one XOR per store)
                sfor<4>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    V w;
                    w.x = d1[c][i] - d2[c][i];
                    w.y = d3[c][i] - d1[c][i] - d2[c][i];
                    lds_put(lds, g_out ^ (swz(toff((uint32_t)i)) * (uint32_t)sizeof(V)), w);
                });
            }
        });
    }
    __builtin_amdgcn_s_setprio(0);
}

template <int K, typename T>
__device__ __forceinline__ void mfma_core(typename CxT<T>::V* lds, int L, const DevOp& op, const MfmaFrag<K, T>& av,
                                          int lane, int wave)
{
    if constexpr (MfmaShape<K, T>::G) {
        mfma_core_gauss<K, T>(lds, L, op, av, lane, wave);
        return;
    } else {
    using V = typename CxT<T>::V;
    using A4 = typename CxT<T>::A4;
    using S = MfmaShape<K, T>;
    constexpr int KS = S::KS, RW = S::RW, CW = S::CW, RPW = S::RPW, CH = S::CH;
    const int rg = wave % RW, cg = wave / RW;
    const int ncb = 1 << (L - K - 4);
    const int nper = (ncb + CW - 1) / CW;      // same for every wave
    uint32_t bit[K];
#pragma unroll
    for (int j = 0; j < K; ++j) bit[j] = 1u << op.pos[j];
    // the 16 columns of a column block differ in the four tile positions of
    // op.c_lane (chosen on the host so that their LDS banks differ); the
    // block number fills the other free positions, op.c_wave
    const uint32_t gl = deposit_bits((uint32_t)(lane & 15), op.c_lane);
    auto toff = [&](uint32_t s) {              // s is a compile-time constant at every call
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (s & (1u << j)) o |= bit[j];
        return o;
    };
    const int krow = lane >> 4;
    const uint32_t in_sw = swz((krow >> 1) ? bit[0] : 0u);                           // bit 0 of s
    const uint32_t out_sw = swz(((krow & 1) ? bit[1] : 0u) | ((krow >> 1) ? bit[2] : 0u));
    const uint32_t part = (uint32_t)(krow & 1);                                       // re / im
    const T* __restrict__ ldsf = reinterpret_cast<const T*>(lds);
    // the wave's column blocks are cg, cg + CW, ...; their free-position bits
    // advance by a masked add (carries pass through the positions outside
    // the mask), one scalar step per block
    const uint32_t wmask = op.c_wave;
    const uint32_t wstep = deposit_bits((uint32_t)CW, wmask);
    uint32_t gblk = deposit_bits((uint32_t)cg, wmask);
    auto mfma = [](const T a, const T b, const A4 c) -> A4 {
        if constexpr (sizeof(T) == 4) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
        else return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    };
    // issue priority over the other work-group's waves on this SIMD while
    // the wave streams MFMAs and writes their results back (the other
    // work-group's tile loads and stores fill the matrix core's gaps instead
    // of delaying it)
    __builtin_amdgcn_s_setprio(1);
    for (int i0 = 0; i0 < nper; i0 += CH) {
        A4 acc[RPW][CH];
        uint32_t gsw[CH], gcol[CH], gin[CH];
        bool ok[CH];
        // CH column blocks at once; a block past the wave's last one reads an
        // in-range column (the masked increment wraps inside the mask) and is
        // not written back, so the loads and MFMAs below need no branches
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            const int blk = cg + (i0 + c) * CW;
            ok[c] = i0 + c < nper && blk < ncb;
#pragma unroll
            for (int r = 0; r < RPW; ++r) acc[r][c] = A4{0, 0, 0, 0};
            gcol[c] = gl | gblk;
            gsw[c] = swz(gcol[c]);
            // byte offset of this lane's (re or im) value: one XOR per load
            gin[c] = (gsw[c] ^ in_sw) * (uint32_t)sizeof(V) + part * (uint32_t)sizeof(T);
            gblk = ((gblk | ~wmask) + wstep) & wmask;
        });
        // B values one k-step ahead of the MFMAs that use them
        T bq[2][CH];
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            bq[0][c] = lds_at(ldsf, gin[c] ^ (swz(toff(0u)) * (uint32_t)sizeof(V)));
        });
        sfor<KS>([&](auto kc) {
            constexpr int ks = decltype(kc)::value;
            constexpr int cur = ks & 1;
            if constexpr (ks + 1 < KS) {
                const uint32_t nx = swz(toff((uint32_t)(2 * (ks + 1)))) * (uint32_t)sizeof(V);
                sfor<CH>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    bq[cur ^ 1][c] = lds_at(ldsf, gin[c] ^ nx);
                });
            }
            // keep the next step's loads ahead of this step's MFMAs (the
            // scheduler would otherwise sink each load next to its use)
            __builtin_amdgcn_sched_barrier(0);
            sfor<CH>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int r = 0; r < RPW; ++r) acc[r][c] = mfma(av[r][ks], bq[cur][c], acc[r][c]);
            });
            __builtin_amdgcn_sched_barrier(0);
        });
        if constexpr (RW > 1) __syncthreads();   // the chunk's B fragments are read
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            if (ok[c] && (gcol[c] & op.c_tile) == op.c_tile) {
                uint32_t g_out = (gsw[c] ^ out_sw) * (uint32_t)sizeof(V);
                asm volatile("" : "+v"(g_out));   // keeps the byte form (one XOR per store)
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    const int rb = rg * RPW + r;
                    const uint32_t o0 = g_out ^ (swz(toff((uint32_t)(8 * rb))) * (uint32_t)sizeof(V));
                    V w0, w1;
                    w0.x = acc[r][c][0];
                    w0.y = acc[r][c][1];
                    w1.x = acc[r][c][2];
                    w1.y = acc[r][c][3];
                    lds_put(lds, o0, w0);
                    lds_put(lds, o0 ^ (swz(bit[0]) * (uint32_t)sizeof(V)), w1);
                }
            }
        });
    }
    __builtin_amdgcn_s_setprio(0);
    }
}

// 32x32x2 three-product form of a complex 2^K x 2^K block on a complex64 LDS
// tile (instantiated for K = 5: a 6-qubit block's fragments would take 96
// registers, which do not fit beside the next tile's prefetch at two
// work-groups per CU).  The block's rows form 2^(K-5) row blocks of 32, one
// per wave of a column group (K = 5: four groups of one wave); a column
// block is 32 columns (groups of 2^K amplitudes), which differ in the five
// tile positions of op.c_lane.  In k-step ks lane l feeds input 2 ks + l/32
// of column l%32 -- one (re, im) read serves the three products T1 = A x,
// T2 = B y, T3 = (A + B)(x + y) -- and the result row 8 (r/4) + 4 (l/32) +
// r%4 of column l%32 comes back in register r.  A fragments: (rb, ks, m)
// lane l holds the m-th part (A, B, A + B) of U[32 rb + l%32][2 ks + l/32],
// either in registers (`ar`, the pass's hoisted block) or read from the
// LDS-staged coefficients one k-step ahead (`al`).  Per k-step the wave
// issues three 64-cycle MFMAs against one LDS read and one add: half the
// other instructions per MFMA cycle of the 16x16x4 form.
template <int K>
struct WideShape {
    static constexpr int KS = 1 << (K - 1);    // k-steps of 2 inputs
    static constexpr int RB = 1 << (K - 5);    // row blocks of 32
    static constexpr int RW = RB;              // waves per column group
    static constexpr int CW = 4 / RW;          // column groups
};
template <int K>
using WideFrag = float[3][WideShape<K>::KS];

using F16 = float __attribute__((ext_vector_type(16)));

template <int K>
__device__ __forceinline__ void wide_load_a(WideFrag<K>& av, const float* __restrict__ A, int lane, int wave)
{
    using S = WideShape<K>;
    const int rb = wave % S::RW;
#pragma unroll
    for (int ks = 0; ks < S::KS; ++ks)
#pragma unroll
        for (int m = 0; m < 3; ++m) av[m][ks] = A[((rb * S::KS + ks) * 3 + m) * 64 + lane];
}

template <int K, int CH, bool AREG>
__device__ __forceinline__ void mfma_core_wide(float2* lds, int L, const DevOp& op, const WideFrag<K>* ar,
                                               const float* __restrict__ al, int lane, int wave)
{
    using S = WideShape<K>;
    constexpr int KS = S::KS, RW = S::RW, CW = S::CW;
    using V = float2;
    const int rb = wave % RW, cg = wave / RW;
    const int ncb = 1 << (L - K - 5);          // the planner keeps ncb a multiple of CW
    const int nper = ncb / CW;
    uint32_t bit[K];
#pragma unroll
    for (int j = 0; j < K; ++j) bit[j] = 1u << op.pos[j];
    auto toff = [&](uint32_t s) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (s & (1u << j)) o |= bit[j];
        return o;
    };
    const uint32_t gl = deposit_bits((uint32_t)(lane & 31), op.c_lane);
    const uint32_t khalf = (uint32_t)(lane >> 5);
    const uint32_t in_sw = swz(khalf ? bit[0] : 0u);
    const uint32_t out_sw = swz(toff(4u * khalf)) ^ swz(toff(32u * (uint32_t)rb));
    const uint32_t wmask = op.c_wave;
    const uint32_t wstep = deposit_bits((uint32_t)CW, wmask);
    uint32_t gblk = deposit_bits((uint32_t)cg, wmask);
    const float* __restrict__ alw = al + (size_t)rb * KS * 3 * 64 + lane;
    __builtin_amdgcn_s_setprio(1);
    for (int i0 = 0; i0 < nper; i0 += CH) {
        F16 d1[CH], d2[CH], d3[CH];
        uint32_t gsw[CH], gcol[CH], gin[CH];
        bool ok[CH];
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            ok[c] = i0 + c < nper;
            gcol[c] = gl | gblk;
            gsw[c] = swz(gcol[c]);
            gin[c] = (gsw[c] ^ in_sw) * (uint32_t)sizeof(V);
            gblk = ((gblk | ~wmask) + wstep) & wmask;
        });
        // inputs, their sums and (LDS-staged blocks) the A fragments one
        // k-step ahead of the MFMAs that use them
        V bq[2][CH];
        float bs[2][CH];
        float aq[2][3];
        auto load_a = [&](auto kc, float* a) {
            constexpr int ks = decltype(kc)::value;
            if constexpr (AREG) {
                a[0] = (*ar)[0][ks];
                a[1] = (*ar)[1][ks];
                a[2] = (*ar)[2][ks];
            } else {
                a[0] = alw[(ks * 3 + 0) * 64];
                a[1] = alw[(ks * 3 + 1) * 64];
                a[2] = alw[(ks * 3 + 2) * 64];
            }
        };
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            bq[0][c] = lds_at(lds, gin[c]);
        });
        load_a(std::integral_constant<int, 0>{}, aq[0]);
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            bs[0][c] = bq[0][c].x + bq[0][c].y;
        });
        sfor<KS>([&](auto kc) {
            constexpr int ks = decltype(kc)::value;
            constexpr int cur = ks & 1;
            if constexpr (ks + 1 < KS) {
                const uint32_t nx = swz(toff((uint32_t)(2 * (ks + 1)))) * (uint32_t)sizeof(V);
                sfor<CH>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    bq[cur ^ 1][c] = lds_at(lds, gin[c] ^ nx);
                });
                if constexpr (!AREG) load_a(std::integral_constant<int, ks + 1>{}, aq[cur ^ 1]);
            }
            if constexpr (AREG) load_a(kc, aq[cur]);
            __builtin_amdgcn_sched_barrier(0);
            sfor<CH>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
                if constexpr (ks == 0) {
                    const F16 z = {};
                    d1[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(aq[cur][0], bq[cur][c].x, z, 0, 0, 0);
                    d2[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(aq[cur][1], bq[cur][c].y, z, 0, 0, 0);
                    d3[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(aq[cur][2], bs[cur][c], z, 0, 0, 0);
                } else {
                    d1[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(aq[cur][0], bq[cur][c].x, d1[c], 0, 0, 0);
                    d2[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(aq[cur][1], bq[cur][c].y, d2[c], 0, 0, 0);
                    d3[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(aq[cur][2], bs[cur][c], d3[c], 0, 0, 0);
                }
            });
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (ks + 1 < KS) {
                sfor<CH>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    bs[cur ^ 1][c] = bq[cur ^ 1][c].x + bq[cur ^ 1][c].y;
                });
                __builtin_amdgcn_sched_barrier(0);
            }
        });
        if constexpr (RW > 1) __syncthreads();   // every wave of the group has read these columns
        sfor<CH>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            if (ok[c] && (gcol[c] & op.c_tile) == op.c_tile) {
                uint32_t g_out = (gsw[c] ^ out_sw) * (uint32_t)sizeof(V);
                asm volatile("" : "+v"(g_out));
                sfor<16>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    constexpr uint32_t row = 8u * (r / 4) + (r % 4);
                    V w;
                    w.x = d1[c][r] - d2[c][r];
                    w.y = d3[c][r] - d1[c][r] - d2[c][r];
                    lds_put(lds, g_out ^ (swz(toff(row)) * (uint32_t)sizeof(V)), w);
                });
            }
        });
    }
    __builtin_amdgcn_s_setprio(0);
}

template <int K, typename T>
__device__ void mfma_lds(typename CxT<T>::V* lds, int L, const DevOp& op, const T* __restrict__ A, int lane,
                         int wave)
{
    MfmaFrag<K, T> av;
    mfma_load_a<K, T>(av, A, lane, wave);
    mfma_core<K, T>(lds, L, op, av, lane, wave);
}

// Matrix-core blocks of at most KMAX qubits (a kernel that keeps a larger
// block's fragments resident dispatches only the small ones here).
// Blocks flagged QOPS_MFMA_WIDE (complex64, 5 qubits) run the 32x32x2 form
// with their fragments read per k-step, WCH column blocks in flight.  WMODE
// says which forms a kernel can meet, so that it compiles only those: 0 =
// never the wide one, 1 = either, 2 = the wide one for every 5-qubit block
// (complex64 on the largest tile).
template <typename T, int KMAX = 6, int WCH = 2, int WMODE = 0>
__device__ void mfma_dispatch(typename CxT<T>::V* lds, int L, const DevOp& op, const T* __restrict__ A, int lane,
                              int wave)
{
    if (op.a > KMAX) return;
    if constexpr (sizeof(T) == 4 && WMODE > 0) {
        if (op.a == 5 && (WMODE == 2 || (op.c_reg & QOPS_MFMA_WIDE))) {
            mfma_core_wide<5, WCH, false>(lds, L, op, nullptr, A, lane, wave);
            return;
        }
    }
    if constexpr (WMODE == 2) {
        switch (op.a) {
        case 3: mfma_lds<3, T>(lds, L, op, A, lane, wave); break;
        case 4: mfma_lds<4, T>(lds, L, op, A, lane, wave); break;
        case 6: if constexpr (KMAX >= 6) mfma_lds<6, T>(lds, L, op, A, lane, wave); break;
        default: break;
        }
        return;
    }
    switch (op.a) {
    case 3: mfma_lds<3, T>(lds, L, op, A, lane, wave); break;
    case 4: mfma_lds<4, T>(lds, L, op, A, lane, wave); break;
    case 5: if constexpr (KMAX >= 5) mfma_lds<5, T>(lds, L, op, A, lane, wave); break;
    case 6: if constexpr (KMAX >= 6) mfma_lds<6, T>(lds, L, op, A, lane, wave); break;
    default: break;
    }
}

// ---------------------------------------------------------------------------
// Tile pass kernel
// ---------------------------------------------------------------------------

template <int R, int W>
struct MapState {
    uint64_t rb[R];     // physical offset of register bit b
    uint32_t lb[R];     // LDS offset of register bit b
    uint64_t tphys;     // physical offset of this thread (lane + wave bits)
    uint32_t tlds;      // LDS offset of this thread
    uint32_t map;
};

template <int R, int W>
__device__ __forceinline__ void set_map(MapState<R, W>& ms, uint32_t map, const int32_t* __restrict__ up_phys, int lane,
                                        int wave)
{
    ms.map = map;
    sfor<R>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        const int u = map_get(map, b);
        ms.rb[b] = 1ull << up_phys[u];
        ms.lb[b] = 1u << (6 + u);
    });
    uint64_t tp = (uint64_t)lane;
    uint32_t tl = (uint32_t)lane;
    sfor<W>([&](auto wc) {
        constexpr int w = decltype(wc)::value;
        const int u = map_get(map, R + w);
        if ((wave >> w) & 1) {
            tp |= 1ull << up_phys[u];
            tl |= 1u << (6 + u);
        }
    });
    ms.tphys = tp;
    ms.tlds = tl;
}

template <int R, int W>
__device__ __forceinline__ uint64_t reg_phys(const MapState<R, W>& ms, int j)
{
    uint64_t o = 0;
    sfor<R>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        if (j & (1 << b)) o |= ms.rb[b];
    });
    return o;
}

template <int R, int W>
__device__ __forceinline__ uint32_t reg_lds(const MapState<R, W>& ms, int j)
{
    uint32_t o = 0;
    sfor<R>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        if (j & (1 << b)) o |= ms.lb[b];
    });
    return o;
}

// One tile of a register-tile pass: load, every operation of the pass,
// store.  `lds` is the work-group's exchange buffer (wave bits), `fresh`
// replaces the load by |0..0> (the first pass of a batched circuit).
template <typename T, int R, int W>
__device__ __forceinline__ void reg_tile(typename CxT<T>::V* __restrict__ st, const PassHdr* __restrict__ hp,
                                         const DevOp* __restrict__ ops, const T* __restrict__ coef, uint64_t tile,
                                         typename CxT<T>::V* lds, int lane, int wave, bool fresh)
{
    using V = typename CxT<T>::V;
    constexpr int NR = 1 << R;
    const int nops = hp->nops;
    const DevOp* __restrict__ prog = ops + hp->op0;
    const int nruns = hp->nruns;
    const int32_t* __restrict__ up_phys = hp->up_phys;
    {
        uint64_t base = 0;
        for (int r = 0; r < nruns; ++r) {
            const uint64_t field = (tile >> hp->run_gshift[r]) & ((1ull << hp->run_len[r]) - 1ull);
            base |= field << hp->run_start[r];
        }
        MapState<R, W> ms;
        set_map<R, W>(ms, (uint32_t)hp->map0, up_phys, lane, wave);
        V a[NR];
        if (fresh) {
            sfor<NR>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                const bool one = base + ms.tphys + reg_phys(ms, j) == 0;
                a[j].x = one ? (T)1 : (T)0;
                a[j].y = (T)0;
            });
        } else {
            const V* src = st + base + ms.tphys;
            sfor<NR>([&](auto jc) { a[decltype(jc)::value] = src[reg_phys(ms, decltype(jc)::value)]; });
        }
        for (int i = 0; i < nops; ++i) {
            const DevOp op = prog[i];
            if ((base & op.c_glob) != op.c_glob) continue;   // tile-uniform control
            switch (op.type) {
            case OP_1Q_REG:
            case OP_1Q_LANE: {
                const T* c = coef + op.coef;
                const V m00 = ldc(c, 0), m01 = ldc(c, 1), m10 = ldc(c, 2), m11 = ldc(c, 3);
                const bool ctrl = (op.c_lane | op.c_wave | op.c_reg) != 0;
                const bool tok = ((uint32_t)lane & op.c_lane) == op.c_lane && ((uint32_t)wave & op.c_wave) == op.c_wave;
                if (op.b == 1) {   // exact X: exchange only
                    if (op.type == OP_1Q_REG) {
                        if (ctrl) xgate_reg<R, true>(op.a, a, op.c_reg, tok);
                        else xgate_reg<R, false>(op.a, a, 0u, true);
                    } else {
                        if (ctrl) xgate_lane<R, true>(op.a, lane, a, op.c_reg, tok);
                        else xgate_lane<R, false>(op.a, lane, a, 0u, true);
                    }
                } else if (op.type == OP_1Q_REG) {
                    if (ctrl)
                        oneq_reg<R, true>(op.a, a, m00, m01, m10, m11, op.c_reg, tok);
                    else
                        oneq_reg<R, false>(op.a, a, m00, m01, m10, m11, 0u, true);
                } else {
                    if (ctrl)
                        oneq_lane<R, true>(op.a, lane, a, m00, m01, m10, m11, op.c_reg, tok);
                    else
                        oneq_lane<R, false>(op.a, lane, a, m00, m01, m10, m11, 0u, true);
                }
                break;
            }
            case OP_CPHASE: {
                // phase on the amplitudes whose masked bits are all 1; the
                // register part of the condition is uniform per slot
                const bool tok = ((uint32_t)lane & op.c_lane) == op.c_lane && ((uint32_t)wave & op.c_wave) == op.c_wave;
                const bool thr = (op.c_lane | op.c_wave) != 0;
                const uint32_t creg = op.c_reg;
                // the multiplier is 1 where the lane's bits do not match
                V ph = ldc(coef + op.coef, 0);
                if (thr) {
                    ph.x = tok ? ph.x : (T)1;
                    ph.y = tok ? ph.y : (T)0;
                }
                if (op.b == 1) {   // -1: flip signs (lanes that do not match multiply by +1)
                    const T sgn = ph.x;
                    sfor<NR>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        if (((uint32_t)j & creg) == creg) {
                            a[j].x *= sgn;
                            a[j].y *= sgn;
                        }
                    });
                } else {
                    sfor<NR>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        if (((uint32_t)j & creg) == creg) a[j] = cmul(a[j], ph);
                    });
                }
                break;
            }
            case OP_DIAG: {
                const T* tab = coef + op.coef;
                const int m = op.a;
                uint32_t ithr = 0;
                uint32_t rm[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    rm[q] = 0;
                    if (q < m) {
                        const int cls = op.pos[q] >> 8, v = op.pos[q] & 255;
                        if (cls == SRC_LANE) ithr |= (uint32_t)((lane >> v) & 1) << q;
                        else if (cls == SRC_WAVE) ithr |= (uint32_t)((wave >> v) & 1) << q;
                        else if (cls == SRC_GLOB) ithr |= (uint32_t)((base >> v) & 1ull) << q;
                        else rm[q] = 1u << v;
                    }
                }
                // table bits held in registers: at most two take the fast path
                // (the four candidate phases are loaded once per thread and
                // selected per slot with uniform conditions)
                int nq = 0, qa = -1, qb = -1;
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    if (rm[q]) {
                        if (nq == 0) qa = q;
                        else if (nq == 1) qb = q;
                        ++nq;
                    }
                if (nq <= 2) {
                    const uint32_t ba = qa >= 0 ? 1u << qa : 0u, bb = qb >= 0 ? 1u << qb : 0u;
                    const uint32_t ma = qa >= 0 ? rm[qa] : 0u, mb = qb >= 0 ? rm[qb] : 0u;
                    V pv[4];
                    pv[0] = ldc(tab, (int)ithr);
                    pv[1] = ldc(tab, (int)(ithr | ba));
                    pv[2] = ldc(tab, (int)(ithr | bb));
                    pv[3] = ldc(tab, (int)(ithr | ba | bb));
                    sfor<NR>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        const int r = (((uint32_t)j & ma) ? 1 : 0) | (((uint32_t)j & mb) ? 2 : 0);   // uniform
                        if (r == 0) a[j] = cmul(a[j], pv[0]);
                        else if (r == 1) a[j] = cmul(a[j], pv[1]);
                        else if (r == 2) a[j] = cmul(a[j], pv[2]);
                        else a[j] = cmul(a[j], pv[3]);
                    });
                } else {
                    sfor<NR>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        uint32_t idx = ithr;
#pragma unroll
                        for (int q = 0; q < 6; ++q)
                            if ((uint32_t)j & rm[q]) idx |= 1u << q;
                        a[j] = cmul(a[j], ldc(tab, (int)idx));
                    });
                }
                break;
            }
            case OP_REMAP:
            case OP_TO_LDS: {
                __syncthreads();
                sfor<NR>([&](auto jc) { lds[ms.tlds + reg_lds(ms, decltype(jc)::value)] = a[decltype(jc)::value]; });
                __syncthreads();
                if (op.type == OP_REMAP) {
                    set_map<R, W>(ms, (uint32_t)op.b, up_phys, lane, wave);
                    sfor<NR>([&](auto jc) { a[decltype(jc)::value] = lds[ms.tlds + reg_lds(ms, decltype(jc)::value)]; });
                }
                break;
            }
            case OP_FROM_LDS: {
                set_map<R, W>(ms, (uint32_t)op.b, up_phys, lane, wave);
                sfor<NR>([&](auto jc) { a[decltype(jc)::value] = lds[ms.tlds + reg_lds(ms, decltype(jc)::value)]; });
                break;
            }
            default:
                break;
            }
        }
        {
            // an opaque copy of the thread offset keeps the compiler from
            // holding every load address live across the operation loop
            uint64_t tp = ms.tphys;
            asm volatile("" : "+v"(tp));
            V* dst = st + base + tp;
            sfor<NR>([&](auto jc) { dst[reg_phys(ms, decltype(jc)::value)] = a[decltype(jc)::value]; });
        }
    }
}

template <typename T, int R, int W>
__global__ void __launch_bounds__(64 << W)
tile_pass_kernel(typename CxT<T>::V* __restrict__ st, const PassHdr* __restrict__ hp, const DevOp* __restrict__ ops,
                 const T* __restrict__ coef, uint64_t ntiles)
{
    using V = typename CxT<T>::V;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        reg_tile<T, R, W>(st, hp, ops, coef, tile, lds, lane, wave, false);
}

// Batched executor: register-tile pass `pass` of every circuit in `items`
// (all planned with the same register/wave split).
template <typename T, int R, int W>
__global__ void __launch_bounds__(64 << W)
batch_reg_kernel(const BatchItem* __restrict__ items, int nitems, const BatchCirc* __restrict__ circs,
                 const PassHdr* __restrict__ hdrs, const DevOp* __restrict__ ops, const T* __restrict__ coef, int pass)
{
    using V = typename CxT<T>::V;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const BatchItem it = items[i];
        const BatchCirc c = circs[it.c];
        reg_tile<T, R, W>(reinterpret_cast<V*>(c.state), hdrs + c.hdr0 + pass, ops, coef, (uint64_t)it.tile, lds,
                          lane, wave, pass == 0);
    }
}

#define QOPS_TILE_VARIANTS(X) \
    X(4, 0) X(4, 1) X(4, 2) X(5, 0) X(5, 1) X(5, 2)

bool tile_variant_supported(int prec, int R, int W)
{
#define QOPS_CHECK(r, w) if (R == r && W == w) return true;
    (void)prec;
    QOPS_TILE_VARIANTS(QOPS_CHECK)
#undef QOPS_CHECK
    return false;
}

int tile_max_lds_bytes() { return 160 * 1024; }

template <typename T, int R, int W>
static hipError_t launch_tile_t(void* state, const PassHdr* hdr, const DevOp* ops, const void* coef, uint64_t ntiles,
                                int lds_bytes, int grid_cap, hipStream_t s)
{
    using V = typename CxT<T>::V;
    auto fn = tile_pass_kernel<T, R, W>;
    static bool attr_done = false;
    if (!attr_done) {
        (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, tile_max_lds_bytes());
        attr_done = true;
    }
    uint64_t grid = ntiles;
    if (grid_cap > 0 && grid > (uint64_t)grid_cap) grid = (uint64_t)grid_cap;
    if (grid > 0x7fffffffull) grid = 0x7fffffffull;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(64 << W), lds_bytes, s, reinterpret_cast<V*>(state), hdr, ops,
                       reinterpret_cast<const T*>(coef), ntiles);
    return hipGetLastError();
}

hipError_t launch_tile_pass(int prec, int R, int W, void* state, const PassHdr* hdr, const DevOp* ops,
                            const void* coef, uint64_t ntiles, int lds_bytes, int grid_cap, hipStream_t s)
{
#define QOPS_LAUNCH(r, w)                                                                              \
    if (R == r && W == w)                                                                              \
        return prec == 0 ? launch_tile_t<float, r, w>(state, hdr, ops, coef, ntiles, lds_bytes, grid_cap, s) \
                         : launch_tile_t<double, r, w>(state, hdr, ops, coef, ntiles, lds_bytes, grid_cap, s);
    QOPS_TILE_VARIANTS(QOPS_LAUNCH)
#undef QOPS_LAUNCH
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// LDS tile pass: the tile (2^L amplitudes, L = 6 + nup) lives in LDS and every
// operation (dense blocks on the vector ALU or matrix cores, diagonals) works
// on it there.  Used for passes that hold dense multi-qubit blocks.
// ---------------------------------------------------------------------------

// Physical offset of upper tile bits v (bit j of v -> physical bit up[j]).
__device__ __forceinline__ uint64_t dep_up(uint32_t v, const int32_t* __restrict__ up, int nup)
{
    uint64_t o = 0;
    for (int j = 0; j < nup; ++j)
        if ((v >> j) & 1u) o |= 1ull << up[j];
    return o;
}

__device__ __forceinline__ uint64_t tile_base(uint64_t tile, const PassHdr* __restrict__ hp)
{
    uint64_t base = 0;
    for (int r = 0; r < hp->nruns; ++r) {
        const uint64_t field = (tile >> hp->run_gshift[r]) & ((1ull << hp->run_len[r]) - 1ull);
        base |= field << hp->run_start[r];
    }
    return base;
}

// Amplitudes per thread of the largest LDS tile (2^13 c64, 2^12 c128).
template <typename T> constexpr int kLdsEpt = sizeof(T) == 4 ? 32 : 16;
template <typename T> constexpr int kLdsTileBytes = sizeof(T) == 4 ? QOPS_LDS_TILE_BYTES_C64 : QOPS_LDS_TILE_BYTES_C128;

// LDS tile pass, persistent and software-pipelined: a work-group stages the
// pass's matrix-core fragments and diagonal tables in LDS once, then loops
// over tiles; while the operations of tile t run on its LDS copy, the loads
// of the next tile are already in flight into registers.  Tile element e has
// physical bits 0..F-1 = e mod 2^F and bit F+j = up_phys[j]
// (F = QOPS_LDS_FIXED_BITS).
// HK > 0: the pass's widest matrix-core block (HK qubits, op hp->hoist) keeps
// its A fragments in registers for every tile of the work-group; the other
// matrix-core blocks of the pass have at most 5 qubits.
// FULL: the tile has the largest size (EPT amplitudes per thread).  Its
// global loads and stores then carry no branch, so the vector-memory counter
// sees one fixed order (the next tile's loads, then this tile's stores) and
// the wait before the LDS fill covers the loads only: the stores drain under
// the next tile's work.  Smaller tiles test each element and wait for all.
template <typename T, int HK, bool FULL>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1)
tile_lds_kernel(typename CxT<T>::V* __restrict__ st, const PassHdr* __restrict__ hp, const DevOp* __restrict__ ops,
                const T* __restrict__ coef, uint64_t ntiles)
{
    using V = typename CxT<T>::V;
    constexpr int EPT = kLdsEpt<T>;
    // one static block at a known LDS address: the swizzled accesses of the
    // matrix-core loops then take one XOR each and no base add
    __shared__ __align__(16) unsigned char smem_raw[kLdsTileBytes<T>];
    V* lds = reinterpret_cast<V*>(smem_raw);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int L = hp->L;
    const int nup = hp->nup;
    const int nops = hp->nops;
    const DevOp* __restrict__ prog = ops + hp->op0;
    const uint32_t N = 1u << L;
    T* lcoef = reinterpret_cast<T*>(smem_raw + ((size_t)N * sizeof(V)));
    {
        const T* __restrict__ src = coef + hp->coef_src;
        for (int i = tid; i < hp->coef_n; i += 256) lcoef[i] = src[i];
    }
    constexpr int HKK = HK > 0 ? HK : 3;
    // the full complex64 tile keeps its hoisted block in the 32x32x2 layout
    // complex64 on the full tile runs its 5-qubit blocks in the 32x32x2 form
    // (a hoisted 5-qubit block keeps that form's fragments)
    constexpr bool WFULL = sizeof(T) == 4 && FULL;
    constexpr bool HWIDE = WFULL && HK == 5;
    MfmaFrag<HKK, T> hav;
    WideFrag<5> haw;
    const int hoist = HK > 0 ? hp->hoist : -1;
    if constexpr (HK > 0) {
        __syncthreads();   // staged coefficients visible
        const DevOp hop = prog[hoist];   // never staged: read from global memory once
        if constexpr (HWIDE) wide_load_a<5>(haw, reinterpret_cast<const float*>(coef) + hop.coef, lane, wave);
        else mfma_load_a<HKK, T>(hav, coef + hop.coef, lane, wave);
    }
    // element e = 256 u + tid: bits 0..F-1 of tid are physical bits 0..F-1
    // (F = QOPS_LDS_FIXED_BITS, contiguous in memory), bits F..7 of tid
    // select up_phys[0 .. 7-F], bit b of u selects up_phys[8-F+b].
    // P2 (full complex64 tiles): each thread moves two adjacent amplitudes
    // with one 16-byte access, element e = 512 u + 2 tid + h: h and bits
    // 0..F-2 of tid are physical bits 0..F-1, bits F-1..7 of tid select
    // up_phys[0 .. 8-F], bit b of u selects up_phys[9-F+b].  Half the vector
    // memory instructions per tile, so a wave's tile stores and the next
    // tile's loads stay within the outstanding-access counter.
    constexpr int F = QOPS_LDS_FIXED_BITS;
    constexpr bool P2 = FULL && sizeof(T) == 4;
    constexpr int NU = P2 ? EPT / 2 : EPT;         // accesses per thread and tile
    constexpr int TB = P2 ? F - 1 : F;              // tid bits inside the contiguous run
    constexpr int UB0 = P2 ? 9 - F : 8 - F;         // up_phys index of u's bit 0
    constexpr int NUB = P2 ? 4 : 5;                 // bits of u
    const uint32_t tlow = ((uint32_t)tid & ((1u << TB) - 1u)) << (P2 ? 1 : 0);
    const uint64_t dep_thr = dep_up((uint32_t)(tid >> TB), hp->up_phys, nup);
    uint64_t ub[NUB];
#pragma unroll
    for (int b = 0; b < NUB; ++b) ub[b] = (UB0 + b < nup) ? (1ull << hp->up_phys[UB0 + b]) : 0ull;
    auto uoff = [&](int u) {
        uint64_t o = 0;
#pragma unroll
        for (int b = 0; b < NUB; ++b)
            if (u & (1 << b)) o += ub[b];
        return o;
    };
    const uint32_t tsw = swz((uint32_t)tid);
    // P2: the pair of element 2 tid (+ 512 u) sits in LDS slots s and s ^ 1 with
    // s = swz(512 u) ^ swz(2 tid); one 16-byte access covers both, in swapped
    // order where bit 0 of swz(2 tid) (= bit 4 of tid) is set
    const uint32_t psw = swz(2u * (uint32_t)tid) & ~1u;
    const bool pswap = (tid >> 4) & 1;
    float4 q2[P2 ? NU : 1];
    T pr[P2 ? 1 : EPT], pi[P2 ? 1 : EPT];
    auto fetch = [&](uint64_t tile) {
        const V* __restrict__ src = st + tile_base(tile, hp) + tlow + dep_thr;
        sfor<NU>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            if constexpr (P2) {
                q2[u] = *reinterpret_cast<const float4*>(src + uoff(u));
            } else if (FULL || 256u * u < N) {
                const V x = src[uoff(u)];
                pr[u] = x.x;
                pi[u] = x.y;
            }
        });
    };
    uint64_t tile = blockIdx.x;
    if (tile < ntiles) fetch(tile);
    // drain the first fetch here, so that the loop head sees outstanding
    // loads from the loop body only
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    for (; tile < ntiles; tile += gridDim.x) {
        const uint64_t base = tile_base(tile, hp);
        sfor<NU>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            if constexpr (P2) {
                const float4 x = q2[u];
                float4 w;
                w.x = pswap ? x.z : x.x;
                w.y = pswap ? x.w : x.y;
                w.z = pswap ? x.x : x.z;
                w.w = pswap ? x.y : x.w;
                lds_put(reinterpret_cast<float4*>(smem_raw), (swz(512u * u) ^ psw) * 8u, w);
            } else if (FULL || 256u * u < N) {
                V x;
                x.x = pr[u];
                x.y = pi[u];
                lds[swz(256u * u) ^ tsw] = x;
            }
        });
        __syncthreads();
        if (tile + gridDim.x < ntiles) fetch(tile + gridDim.x);
        for (int i = 0; i < nops; ++i) {
            const DevOp op = prog[i];
            if ((base & op.c_glob) != op.c_glob) continue;
            // complex64 passes hold every coefficient except the hoisted
            // block's in LDS (the planner guarantees it), so their ops issue
            // no vector-memory loads and never wait on the next tile's loads
            // in flight; complex128 ops read from LDS (op.b = 1) or global
            const T* cf;
            if constexpr (sizeof(T) == 4) cf = lcoef + op.coef;
            else cf = op.b ? lcoef + op.coef : coef + op.coef;
            if (op.type == OP_DENSE_LDS) {
                dense_lds_dispatch<T>(lds, L, op, cf, tid, 256);
            } else if (op.type == OP_MFMA) {
                if constexpr (HWIDE) {
                    if (i == hoist) mfma_core_wide<5, 1, true>(lds, L, op, &haw, nullptr, lane, wave);
                    else mfma_dispatch<T, 5, 1, 2>(lds, L, op, cf, lane, wave);
                } else if constexpr (WFULL && HK > 0) {
                    // beside a hoisted 6-qubit block, one column block of the
                    // 5-qubit ones in flight
                    if (i == hoist) mfma_core<HKK, T>(lds, L, op, hav, lane, wave);
                    else mfma_dispatch<T, 5, 1, 2>(lds, L, op, cf, lane, wave);
                } else if constexpr (HK > 0) {
                    if (i == hoist) mfma_core<HKK, T>(lds, L, op, hav, lane, wave);
                    else mfma_dispatch<T, 5>(lds, L, op, cf, lane, wave);
                } else if constexpr (WFULL) {
                    mfma_dispatch<T, 6, 2, 2>(lds, L, op, cf, lane, wave);
                } else {
                    mfma_dispatch<T>(lds, L, op, cf, lane, wave);
                }
            } else if (op.type == OP_DIAG_LDS) {
                diag_lds<T>(lds, L, op, cf, base, tid, 256);
            }
            __syncthreads();
        }
        {
            V* __restrict__ dst = st + base + tlow + dep_thr;
            sfor<NU>([&](auto uc) {
                constexpr int u = decltype(uc)::value;
                if constexpr (P2) {
                    const float4 x = lds_at(reinterpret_cast<const float4*>(smem_raw), (swz(512u * u) ^ psw) * 8u);
                    float4 w;
                    w.x = pswap ? x.z : x.x;
                    w.y = pswap ? x.w : x.y;
                    w.z = pswap ? x.x : x.z;
                    w.w = pswap ? x.y : x.w;
                    *reinterpret_cast<float4*>(dst + uoff(u)) = w;
                } else if (FULL || 256u * u < N) {
                    dst[uoff(u)] = lds[swz(256u * u) ^ tsw];
                }
            });
        }
        __syncthreads();
    }
}

static int g_num_cus = 0;

static int num_cus()
{
    if (g_num_cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            g_num_cus = v;
        else
            g_num_cus = 256;
    }
    return g_num_cus;
}

template <typename T, int HK, bool FULL>
static hipError_t launch_tile_lds_f(void* state, const PassHdr* hdr, const DevOp* ops, const void* coef,
                                    uint64_t grid, uint64_t ntiles, int lds_bytes, hipStream_t s)
{
    using V = typename CxT<T>::V;
    (void)lds_bytes;   // checked against the kernel's static block by the caller
    hipLaunchKernelGGL((tile_lds_kernel<T, HK, FULL>), dim3((unsigned)grid), dim3(256), 0, s,
                       reinterpret_cast<V*>(state), hdr, ops, reinterpret_cast<const T*>(coef), ntiles);
    return hipGetLastError();
}

template <typename T, int HK>
static hipError_t launch_tile_lds_t(void* state, const PassHdr* hdr, const DevOp* ops, const void* coef,
                                    uint64_t grid, uint64_t ntiles, int L, int lds_bytes, hipStream_t s)
{
    constexpr int LMAX = sizeof(T) == 4 ? 13 : 12;   // 256 threads x kLdsEpt<T>
    if (L == LMAX) return launch_tile_lds_f<T, HK, true>(state, hdr, ops, coef, grid, ntiles, lds_bytes, s);
    return launch_tile_lds_f<T, HK, false>(state, hdr, ops, coef, grid, ntiles, lds_bytes, s);
}

hipError_t launch_tile_lds(int prec, void* state, const PassHdr* hdr, const DevOp* ops, const void* coef,
                           uint64_t ntiles, int L, int lds_bytes, int grid_cap, int hoist_k, hipStream_t s)
{
    // persistent grid: as many work-groups as fit on the chip (the kernel's
    // static LDS block; the planner keeps tile plus coefficients within it)
    const int block = prec == 0 ? QOPS_LDS_TILE_BYTES_C64 : QOPS_LDS_TILE_BYTES_C128;
    if (lds_bytes > block) return hipErrorInvalidValue;
    const int per_cu = std::max(1, tile_max_lds_bytes() / block);
    uint64_t grid = std::min<uint64_t>(ntiles, (uint64_t)num_cus() * per_cu);
    if (grid_cap > 0 && grid > (uint64_t)grid_cap) grid = (uint64_t)grid_cap;
    if (grid == 0) grid = 1;
    if (prec == 0) {
        if (hoist_k == 6) return launch_tile_lds_t<float, 6>(state, hdr, ops, coef, grid, ntiles, L, lds_bytes, s);
        if (hoist_k == 5) return launch_tile_lds_t<float, 5>(state, hdr, ops, coef, grid, ntiles, L, lds_bytes, s);
        return launch_tile_lds_t<float, 0>(state, hdr, ops, coef, grid, ntiles, L, lds_bytes, s);
    }
    return launch_tile_lds_t<double, 0>(state, hdr, ops, coef, grid, ntiles, L, lds_bytes, s);
}

// ---------------------------------------------------------------------------
// Whole state in one work-group's LDS
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void run_ops_lds(typename CxT<T>::V* lds, int n, const DevOp* __restrict__ ops, int nops,
                           const T* __restrict__ coef, int tid, int nthr)
{
    const int lane = tid & 63, wave = tid >> 6;
    // diagonal tables (<= 64 entries) are copied to LDS first: their lookups
    // are data dependent, and from global memory each one would wait on L2
    __shared__ __align__(16) T ctab[2 * 64];
    for (int i = 0; i < nops; ++i) {
        const DevOp op = ops[i];
        if (op.type == OP_DENSE_LDS) {
            dense_lds_dispatch<T>(lds, n, op, coef + op.coef, tid, nthr);
        } else if (op.type == OP_MFMA) {
            mfma_dispatch<T>(lds, n, op, coef + op.coef, lane, wave);
        } else if (op.type == OP_DIAG_LDS) {
            const int cnt = 2 << op.a;
            for (int j = tid; j < cnt; j += nthr) ctab[j] = coef[op.coef + j];
            __syncthreads();
            diag_lds<T>(lds, n, op, ctab, 0ull, tid, nthr);
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
state_lds_kernel(typename CxT<T>::V* __restrict__ st, int n, const DevOp* __restrict__ ops, int nops,
                 const T* __restrict__ coef)
{
    using V = typename CxT<T>::V;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    const uint32_t N = 1u << n;
    for (uint32_t x = threadIdx.x; x < N; x += blockDim.x) lds[swz(x)] = st[x];
    __syncthreads();
    run_ops_lds<T>(lds, n, ops, nops, coef, threadIdx.x, blockDim.x);
    for (uint32_t x = threadIdx.x; x < N; x += blockDim.x) st[x] = lds[swz(x)];
}

hipError_t launch_state_lds(int prec, void* state, int n, const DevOp* ops, int nops, const void* coef,
                            hipStream_t s)
{
    const size_t bytes = (size_t(1) << n) * (prec == 0 ? 8 : 16);
    if (prec == 0) {
        if (hipError_t e = hipFuncSetAttribute((const void*)state_lds_kernel<float>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))
            return e;
        hipLaunchKernelGGL(state_lds_kernel<float>, dim3(1), dim3(256), bytes, s, reinterpret_cast<float2*>(state), n,
                           ops, nops, reinterpret_cast<const float*>(coef));
    } else {
        if (hipError_t e = hipFuncSetAttribute((const void*)state_lds_kernel<double>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))
            return e;
        hipLaunchKernelGGL(state_lds_kernel<double>, dim3(1), dim3(256), bytes, s, reinterpret_cast<double2*>(state),
                           n, ops, nops, reinterpret_cast<const double*>(coef));
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gate-wise HBM sweep (one operation per launch; the unfused simulator)
// ---------------------------------------------------------------------------

template <typename T, int K>
__global__ void __launch_bounds__(256)
sweep_dense_kernel(typename CxT<T>::V* __restrict__ st, uint64_t ngroups, uint64_t tmask, uint64_t cmask,
                   int4 p03, int2 p45, const T* __restrict__ U)
{
    using V = typename CxT<T>::V;
    constexpr int D = 1 << K;
    const int pos[6] = {p03.x, p03.y, p03.z, p03.w, p45.x, p45.y};
    uint64_t toff[D];
#pragma unroll
    for (int s = 0; s < D; ++s) {
        uint64_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (s & (1 << j)) o |= 1ull << pos[j];
        toff[s] = o;
    }
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < ngroups;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = spread_mask64(g, tmask);
        if ((x & cmask) != cmask) continue;
        V in[D];
#pragma unroll
        for (int s = 0; s < D; ++s) in[s] = st[x + toff[s]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            V acc;
            acc.x = 0;
            acc.y = 0;
#pragma unroll
            for (int s = 0; s < D; ++s) {
                const T ur = U[2 * (r * D + s)], ui = U[2 * (r * D + s) + 1];
                acc.x += ur * in[s].x - ui * in[s].y;
                acc.y += ur * in[s].y + ui * in[s].x;
            }
            st[x + toff[r]] = acc;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
sweep_diag_kernel(typename CxT<T>::V* __restrict__ st, uint64_t N, int m, int4 p03, int2 p45, const T* __restrict__ tab)
{
    const int pos[6] = {p03.x, p03.y, p03.z, p03.w, p45.x, p45.y};
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < N; x += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t idx = 0;
        for (int i = 0; i < m; ++i) idx |= (uint32_t)((x >> pos[i]) & 1ull) << i;
        st[x] = cmul(st[x], ldc(tab, (int)idx));
    }
}

static unsigned grid_for(uint64_t work, unsigned block, int grid_cap = 0)
{
    uint64_t g = (work + block - 1) / block;
    const uint64_t cap = 256ull * 64;   // enough waves to fill 256 CUs, grid-stride beyond
    if (g > cap) g = cap;
    if (grid_cap > 0 && g > (uint64_t)grid_cap) g = (uint64_t)grid_cap;
    if (g == 0) g = 1;
    return (unsigned)g;
}

template <typename T>
static hipError_t launch_sweep_t(void* state, int n, const DevOp* op, const void* coef, int grid_cap, hipStream_t s)
{
    using V = typename CxT<T>::V;
    V* st = reinterpret_cast<V*>(state);
    const T* c = reinterpret_cast<const T*>(coef) + op->coef;
    const int4 p03 = make_int4(op->pos[0], op->pos[1], op->pos[2], op->pos[3]);
    const int2 p45 = make_int2(op->pos[4], op->pos[5]);
    if (op->type == OP_DIAG_LDS) {
        const uint64_t N = 1ull << n;
        hipLaunchKernelGGL(sweep_diag_kernel<T>, dim3(grid_for(N, 256, grid_cap)), dim3(256), 0, s, st, N, op->a, p03, p45,
                           c);
        return hipGetLastError();
    }
    const int k = op->a;
    uint64_t tmask = 0;
    for (int j = 0; j < k; ++j) tmask |= 1ull << op->pos[j];
    const uint64_t cmask = op->c_glob;
    const uint64_t ng = 1ull << (n - k);
    const dim3 grid(grid_for(ng, 256, grid_cap)), blk(256);
    switch (k) {
    case 1: hipLaunchKernelGGL((sweep_dense_kernel<T, 1>), grid, blk, 0, s, st, ng, tmask, cmask, p03, p45, c); break;
    case 2: hipLaunchKernelGGL((sweep_dense_kernel<T, 2>), grid, blk, 0, s, st, ng, tmask, cmask, p03, p45, c); break;
    case 3: hipLaunchKernelGGL((sweep_dense_kernel<T, 3>), grid, blk, 0, s, st, ng, tmask, cmask, p03, p45, c); break;
    case 4: hipLaunchKernelGGL((sweep_dense_kernel<T, 4>), grid, blk, 0, s, st, ng, tmask, cmask, p03, p45, c); break;
    case 5: hipLaunchKernelGGL((sweep_dense_kernel<T, 5>), grid, blk, 0, s, st, ng, tmask, cmask, p03, p45, c); break;
    case 6: hipLaunchKernelGGL((sweep_dense_kernel<T, 6>), grid, blk, 0, s, st, ng, tmask, cmask, p03, p45, c); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep(int prec, void* state, int n, const DevOp* op_host, const void* coef_dev, int grid_cap,
                        hipStream_t s)
{
    return prec == 0 ? launch_sweep_t<float>(state, n, op_host, coef_dev, grid_cap, s)
                     : launch_sweep_t<double>(state, n, op_host, coef_dev, grid_cap, s);
}

// ---------------------------------------------------------------------------
// Bit exchange (physical SWAP) and basis initialisation
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256)
swap_bits_kernel(typename CxT<T>::V* __restrict__ st, uint64_t ng, uint64_t mask2, uint64_t ma, uint64_t mb)
{
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < ng; g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x0 = spread_mask64(g, mask2) | ma;   // bit a = 1, bit b = 0
        const uint64_t x1 = x0 ^ ma ^ mb;                  // bit a = 0, bit b = 1
        const auto v0 = st[x0];
        const auto v1 = st[x1];
        st[x0] = v1;
        st[x1] = v0;
    }
}

hipError_t launch_swap_bits(int prec, void* state, int n, int a, int b, int grid_cap, hipStream_t s)
{
    const uint64_t ng = 1ull << (n - 2);
    const uint64_t ma = 1ull << a, mb = 1ull << b;
    if (prec == 0)
        hipLaunchKernelGGL(swap_bits_kernel<float>, dim3(grid_for(ng, 256, grid_cap)), dim3(256), 0, s,
                           reinterpret_cast<float2*>(state), ng, ma | mb, ma, mb);
    else
        hipLaunchKernelGGL(swap_bits_kernel<double>, dim3(grid_for(ng, 256, grid_cap)), dim3(256), 0, s,
                           reinterpret_cast<double2*>(state), ng, ma | mb, ma, mb);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) init_basis_kernel(typename CxT<T>::V* __restrict__ st, uint64_t N, uint64_t x0)
{
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < N; x += (uint64_t)gridDim.x * blockDim.x) {
        typename CxT<T>::V v;
        v.x = (x == x0) ? (T)1 : (T)0;
        v.y = 0;
        st[x] = v;
    }
}

hipError_t launch_init_basis(int prec, void* state, int n, uint64_t x, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    if (prec == 0)
        hipLaunchKernelGGL(init_basis_kernel<float>, dim3(grid_for(N, 256)), dim3(256), 0, s,
                           reinterpret_cast<float2*>(state), N, x);
    else
        hipLaunchKernelGGL(init_basis_kernel<double>, dim3(grid_for(N, 256)), dim3(256), 0, s,
                           reinterpret_cast<double2*>(state), N, x);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 reductions (fixed order, so results are bitwise reproducible)
// ---------------------------------------------------------------------------

template <typename V>
__device__ __forceinline__ double prob(V v)
{
    const double re = (double)v.x, im = (double)v.y;
    return re * re + im * im;
}

// Tree sum over the 256 threads of a block, fixed order.  `sh` has 256 doubles.
__device__ __forceinline__ double block_sum_256(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Block b sums the chunk [b 2^s, (b+1) 2^s): part[b*(n+1) + 0] = sum p,
// part[b*(n+1) + 1 + q] = sum p * bit_q(x).  Bits 8..s-1 of x come from the
// loop counter; LB >= s - 8 of them are tracked in registers.
template <typename T, int LB>
__global__ void __launch_bounds__(256)
zsum_part_kernel(const typename CxT<T>::V* __restrict__ st, int n, int s, double* __restrict__ part)
{
    __shared__ double sh[256];
    const uint64_t base = (uint64_t)blockIdx.x << s;
    const uint32_t chunk = 1u << s;
    const int t = threadIdx.x;
    const int jb = s > 8 ? s - 8 : 0;           // bits 8..s-1 come from the loop counter
    double tot = 0.0;
    double sb[LB];
#pragma unroll
    for (int q = 0; q < LB; ++q) sb[q] = 0.0;
    for (uint32_t j = 0; (j << 8) < chunk; ++j) {
        const uint32_t off = (j << 8) + t;
        if (off >= chunk) break;
        const double p = prob(st[base + off]);
        tot += p;
#pragma unroll
        for (int q = 0; q < LB; ++q)
            if (q < jb && ((j >> q) & 1u)) sb[q] += p;
    }
    double* out = part + (uint64_t)blockIdx.x * (n + 1);
    const double all = block_sum_256(tot, sh);
    if (t == 0) out[0] = all;
    for (int q = 0; q < n; ++q) {
        double v;
        if (q < 8 && q < s)
            v = block_sum_256(((t >> q) & 1) ? tot : 0.0, sh);
        else if (q < s) {
            double mine = 0.0;
#pragma unroll
            for (int r = 0; r < LB; ++r)
                if (r == q - 8) mine = sb[r];
            v = block_sum_256(mine, sh);
        }
        else
            v = ((base >> q) & 1ull) ? all : 0.0;
        if (t == 0) out[1 + q] = v;
    }
}

// One block per output quantity: sums part[b*(n+1) + qi] over blocks b.
__global__ void __launch_bounds__(256) zsum_final_kernel(const double* __restrict__ part, int nparts, int n,
                                                         double* __restrict__ out)
{
    __shared__ double sh[256];
    const int qi = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nparts; b += 256) v += part[(uint64_t)b * (n + 1) + qi];
    const double r = block_sum_256(v, sh);
    if (threadIdx.x == 0) out[qi] = r;
}

static int zsum_chunk_bits(int n) { return n < 16 ? n : 16; }

size_t zsum_scratch_doubles(int n)
{
    const int s = zsum_chunk_bits(n);
    return (size_t(1) << (n - s)) * (n + 1);
}

template <typename T>
static void launch_zsum_part(const void* state, int n, int s, double* part, hipStream_t st)
{
    using V = typename CxT<T>::V;
    const unsigned nb = 1u << (n - s);
    if (s <= 16)
        hipLaunchKernelGGL((zsum_part_kernel<T, 8>), dim3(nb), dim3(256), 0, st, reinterpret_cast<const V*>(state), n,
                           s, part);
    else
        hipLaunchKernelGGL((zsum_part_kernel<T, 16>), dim3(nb), dim3(256), 0, st, reinterpret_cast<const V*>(state),
                           n, s, part);
}

static hipError_t launch_zsum_s(int prec, const void* state, int n, int s, double* part, double* out, hipStream_t st)
{
    if (prec == 0) launch_zsum_part<float>(state, n, s, part, st);
    else launch_zsum_part<double>(state, n, s, part, st);
    hipLaunchKernelGGL(zsum_final_kernel, dim3(n + 1), dim3(256), 0, st, part, (int)(1u << (n - s)), n, out);
    return hipGetLastError();
}

hipError_t launch_zsum(int prec, const void* state, int n, double* scratch, double* out, hipStream_t st)
{
    return launch_zsum_s(prec, state, n, zsum_chunk_bits(n), scratch, out, st);
}

// Chunks of 2^s amplitudes with s = max(zsum_chunk_bits(n), n - 11): at
// most 2^11 partial records whatever n is (up to 24 chunk bits at n = 34);
// for n <= 27 the chunks, and so the summation order, equal launch_zsum's.
static int zsum_bounded_chunk_bits(int n) { return std::max(zsum_chunk_bits(n), n - 11); }

size_t zsum_bounded_scratch_doubles(int n)
{
    return (size_t(1) << (n - zsum_bounded_chunk_bits(n))) * (n + 1) + (n + 1);
}

// out[q] = sums[0] - 2 sums[1 + l2p[q]]: <Z_q> of logical qubit q.
__global__ void z_logical_kernel(const double* __restrict__ sums, int n, ZLayout lay, double* __restrict__ out)
{
    const int q = threadIdx.x;
    if (q < n) out[q] = sums[0] - 2.0 * sums[1 + lay.l2p[q]];
}

hipError_t launch_expect_z_bounded(int prec, const void* state, int n, const int32_t* l2p, double* scratch,
                                   double* out, hipStream_t st)
{
    if (n < 1 || n > QOPS_MAX_QUBITS_DEV) return hipErrorInvalidValue;
    const int s = zsum_bounded_chunk_bits(n);
    double* part = scratch;
    double* sums = scratch + (size_t(1) << (n - s)) * (n + 1);
    hipError_t e = launch_zsum_s(prec, state, n, s, part, sums, st);
    if (e != hipSuccess) return e;
    ZLayout lay;
    for (int q = 0; q < QOPS_MAX_QUBITS_DEV; ++q) lay.l2p[q] = q < n ? l2p[q] : 0;
    hipLaunchKernelGGL(z_logical_kernel, dim3(1), dim3(64), 0, st, sums, n, lay, out);
    return hipGetLastError();
}

// Marginal probabilities.  Three paths:
//  (a) m == n: a permutation of |psi|^2, no reduction;
//  (b) at most 12 marginal bits: block b owns the chunk [b 2^s, (b+1) 2^s),
//      reduces it sub-chunk by sub-chunk (4096 amplitudes) in LDS with a
//      fixed summation order, and writes 2^(marginal bits below s) partials;
//      a second kernel sums the partials over blocks in block order;
//  (c) otherwise one thread per output y sums its 2^(n-m) terms in order.
struct ProbGeom {
    int s;          // chunk bits
    int m_lo;       // marginal bits below s
    int m12;        // marginal bits below 12
    uint32_t lo_mask;  // physical mask of marginal bits below s
};

static ProbGeom prob_geom(int n, int m, const int* pos)
{
    ProbGeom g;
    g.s = n < 20 ? n : 20;
    g.m_lo = 0;
    g.m12 = 0;
    g.lo_mask = 0;
    for (int j = 0; j < m; ++j) {
        if (pos[j] < g.s) {
            g.m_lo++;
            g.lo_mask |= 1u << pos[j];
        }
        if (pos[j] < 12) g.m12++;
    }
    return g;
}

struct PosArr {
    int p[QOPS_MAX_QUBITS_DEV];
};

template <typename T>
__global__ void __launch_bounds__(256)
probs_direct_kernel(const typename CxT<T>::V* __restrict__ st, int n, PosArr pa, double* __restrict__ out)
{
    const uint64_t N = 1ull << n;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < N; x += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t y = 0;
        for (int j = 0; j < n; ++j) y |= ((x >> pa.p[j]) & 1ull) << j;
        out[y] = prob(st[x]);
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
probs_slow_kernel(const typename CxT<T>::V* __restrict__ st, int n, int m, PosArr pa, uint64_t pmask,
                  double* __restrict__ out)
{
    const uint64_t ny = 1ull << m;
    const uint64_t nz = 1ull << (n - m);
    for (uint64_t y = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; y < ny; y += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t xy = 0;
        for (int j = 0; j < m; ++j) xy |= ((y >> j) & 1ull) << pa.p[j];
        double acc = 0.0;
        for (uint64_t z = 0; z < nz; ++z) acc += prob(st[xy | spread_mask64(z, pmask)]);
        out[y] = acc;
    }
}

// y index of x restricted to the marginal bits selected by `sel` (a subset of
// the m marginal bits, in j order), compressed.
__device__ __forceinline__ uint32_t compress_sel(uint64_t x, const PosArr& pa, int m, uint32_t sel)
{
    uint32_t y = 0;
    int o = 0;
    for (int j = 0; j < m; ++j)
        if (sel & (1u << j)) {
            y |= (uint32_t)((x >> pa.p[j]) & 1ull) << o;
            ++o;
        }
    return y;
}

template <typename T>
__global__ void __launch_bounds__(256)
probs_part_kernel(const typename CxT<T>::V* __restrict__ st, int m, PosArr pa, int s, int m_lo,
                  uint32_t sel_lo, uint32_t sel12, int m12, uint32_t mask12, double* __restrict__ part)
{
    __shared__ double tab[4096];
    __shared__ double acc[4096];
    const int t = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x << s;
    const uint32_t nacc = 1u << m_lo;
    for (uint32_t i = t; i < nacc; i += 256) acc[i] = 0.0;
    const int sub_bits = s < 12 ? s : 12;
    const uint32_t sub = 1u << sub_bits;
    const uint32_t nsub = 1u << (s - sub_bits);
    const uint32_t n12 = 1u << m12;
    const uint32_t nz = 1u << (sub_bits - m12);
    __syncthreads();
    for (uint32_t c = 0; c < nsub; ++c) {
        const uint64_t sb = base + (uint64_t)c * sub;
        for (uint32_t i = t; i < sub; i += 256) tab[i] = prob(st[sb + i]);
        __syncthreads();
        for (uint32_t y12 = t; y12 < n12; y12 += 256) {
            // scatter y12 into the marginal bits below 12 (j order)
            uint32_t xy = 0;
            int o = 0;
            for (int j = 0; j < m; ++j)
                if (sel12 & (1u << j)) {
                    xy |= ((y12 >> o) & 1u) << pa.p[j];
                    ++o;
                }
            double v = 0.0;
            for (uint32_t z = 0; z < nz; ++z) v += tab[xy | spread_mask(z, mask12)];
            const uint32_t slot = compress_sel(sb | xy, pa, m, sel_lo);
            acc[slot] += v;
        }
        __syncthreads();
    }
    for (uint32_t i = t; i < nacc; i += 256) part[(uint64_t)blockIdx.x * nacc + i] = acc[i];
}

template <typename T>
__global__ void __launch_bounds__(256)
probs_reduce_kernel(const double* __restrict__ part, int n, int m, PosArr pa, int s, int m_lo, uint32_t sel_lo,
                    uint64_t hi_mask_blocks, double* __restrict__ out)
{
    // hi_mask_blocks: bits of the block number that are marginal bits
    const uint32_t ny = 1u << m;
    const uint32_t nacc = 1u << m_lo;
    const int nbb = n - s;
    const uint64_t nfree = 1ull << (nbb - __popcll(hi_mask_blocks));
    for (uint32_t y = blockIdx.x * blockDim.x + threadIdx.x; y < ny; y += gridDim.x * blockDim.x) {
        uint32_t ylo = 0, o = 0;
        uint64_t bfix = 0;
        for (int j = 0; j < m; ++j) {
            const uint32_t bit = (y >> j) & 1u;
            if (sel_lo & (1u << j)) {
                ylo |= bit << o;
                ++o;
            } else {
                bfix |= (uint64_t)bit << (pa.p[j] - s);
            }
        }
        double v = 0.0;
        for (uint64_t f = 0; f < nfree; ++f) {
            const uint64_t b = bfix | spread_mask64(f, hi_mask_blocks);
            v += part[b * nacc + ylo];
        }
        out[y] = v;
    }
}

size_t probs_scratch_doubles(int n, int m, const int* pos)
{
    if (m == n || m > 12) return 0;
    const ProbGeom g = prob_geom(n, m, pos);
    return (size_t(1) << (n - g.s)) * (size_t(1) << g.m_lo);
}

hipError_t launch_probs(int prec, const void* state, int n, int m, const int* pos, double* scratch, double* out,
                        hipStream_t st)
{
    PosArr pa;
    for (int j = 0; j < QOPS_MAX_QUBITS_DEV; ++j) pa.p[j] = j < m ? pos[j] : 0;
    uint64_t pmask = 0;
    for (int j = 0; j < m; ++j) pmask |= 1ull << pos[j];
    if (m == n) {
        const uint64_t N = 1ull << n;
        if (prec == 0)
            hipLaunchKernelGGL(probs_direct_kernel<float>, dim3(grid_for(N, 256)), dim3(256), 0, st,
                               reinterpret_cast<const float2*>(state), n, pa, out);
        else
            hipLaunchKernelGGL(probs_direct_kernel<double>, dim3(grid_for(N, 256)), dim3(256), 0, st,
                               reinterpret_cast<const double2*>(state), n, pa, out);
        return hipGetLastError();
    }
    if (m > 12) {
        const uint64_t ny = 1ull << m;
        if (prec == 0)
            hipLaunchKernelGGL(probs_slow_kernel<float>, dim3(grid_for(ny, 256)), dim3(256), 0, st,
                               reinterpret_cast<const float2*>(state), n, m, pa, pmask, out);
        else
            hipLaunchKernelGGL(probs_slow_kernel<double>, dim3(grid_for(ny, 256)), dim3(256), 0, st,
                               reinterpret_cast<const double2*>(state), n, m, pa, pmask, out);
        return hipGetLastError();
    }
    const ProbGeom g = prob_geom(n, m, pos);
    uint32_t sel_lo = 0, sel12 = 0, mask12 = 0;
    uint64_t hi_blocks = 0;
    for (int j = 0; j < m; ++j) {
        if (pos[j] < g.s) sel_lo |= 1u << j;
        else hi_blocks |= 1ull << (pos[j] - g.s);
        if (pos[j] < 12 && pos[j] < g.s) {
            sel12 |= 1u << j;
            mask12 |= 1u << pos[j];
        }
    }
    int m12 = __builtin_popcount(sel12);
    const unsigned nb = 1u << (n - g.s);
    if (prec == 0)
        hipLaunchKernelGGL(probs_part_kernel<float>, dim3(nb), dim3(256), 0, st, reinterpret_cast<const float2*>(state),
                           m, pa, g.s, g.m_lo, sel_lo, sel12, m12, mask12, scratch);
    else
        hipLaunchKernelGGL(probs_part_kernel<double>, dim3(nb), dim3(256), 0, st,
                           reinterpret_cast<const double2*>(state), m, pa, g.s, g.m_lo, sel_lo, sel12, m12, mask12,
                           scratch);
    const uint64_t ny = 1ull << m;
    hipLaunchKernelGGL(probs_reduce_kernel<float>, dim3(grid_for(ny, 256)), dim3(256), 0, st, scratch, n, m, pa, g.s,
                       g.m_lo, sel_lo, hi_blocks, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Logical-order gather (readout through the layout map)
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256)
gather_logical_kernel(const typename CxT<T>::V* __restrict__ st, int n, PosArr l2p, uint64_t x0, uint64_t count,
                      typename CxT<T>::V* __restrict__ dst)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = x0 + i;
        uint64_t p = 0;
        for (int q = 0; q < n; ++q) p |= ((x >> q) & 1ull) << l2p.p[q];
        dst[i] = st[p];
    }
}

hipError_t launch_gather_logical(int prec, const void* state, int n, const int* l2p, uint64_t x0, uint64_t count,
                                 void* dst, hipStream_t s)
{
    PosArr pa;
    for (int j = 0; j < QOPS_MAX_QUBITS_DEV; ++j) pa.p[j] = j < n ? l2p[j] : 0;
    if (prec == 0)
        hipLaunchKernelGGL(gather_logical_kernel<float>, dim3(grid_for(count, 256)), dim3(256), 0, s,
                           reinterpret_cast<const float2*>(state), n, pa, x0, count, reinterpret_cast<float2*>(dst));
    else
        hipLaunchKernelGGL(gather_logical_kernel<double>, dim3(grid_for(count, 256)), dim3(256), 0, s,
                           reinterpret_cast<const double2*>(state), n, pa, x0, count, reinterpret_cast<double2*>(dst));
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Batched executor (many small circuits, one graph launch)
// ---------------------------------------------------------------------------

// Fixed-order sum over the 256 threads of a block of v; every thread gets it.
__device__ __forceinline__ double bsum(double v, double* sh)
{
    return block_sum_256(v, sh);
}

// One work-group per circuit whose whole state fits in LDS: |0..0>, every
// operation, then <Z_q> = sum p - 2 sum_{x: bit q} p, reduced in FP64.
template <typename T>
__global__ void __launch_bounds__(256)
batch_small_kernel(const int32_t* __restrict__ ids, const BatchCirc* __restrict__ circs, const DevOp* __restrict__ ops,
                   const T* __restrict__ coef, double* __restrict__ out)
{
    using V = typename CxT<T>::V;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double sh[256];
    V* lds = reinterpret_cast<V*>(smem_raw);
    const BatchCirc c = circs[ids[blockIdx.x]];
    const int n = c.n;
    const uint32_t N = 1u << n;
    const int tid = threadIdx.x;
    for (uint32_t x = tid; x < N; x += 256) {
        V v;
        v.x = x == 0 ? (T)1 : (T)0;
        v.y = 0;
        lds[swz(x)] = v;
    }
    __syncthreads();
    run_ops_lds<T>(lds, n, ops + c.op0, c.nops, coef, tid, 256);
    // one sweep over the LDS state per output (q = -1: the total)
    double all = 0.0;
    for (int q = -1; q < n; ++q) {
        double acc = 0.0;
        for (uint32_t x = tid; x < N; x += 256) {
            if (q >= 0 && !((x >> q) & 1u)) continue;
            const V v = lds[swz(x)];
            acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
        const double s = bsum(acc, sh);
        if (q < 0) all = s;
        else if (tid == 0) out[c.out0 + q] = all - 2.0 * s;
    }
}

// Pass `pass` of every circuit that has one: grid-stride over its tiles.
// Pass 0 starts from |0..0> instead of reading the state.
template <typename T>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1)
batch_pass_kernel(const BatchItem* __restrict__ items, int nitems, const BatchCirc* __restrict__ circs,
                  const PassHdr* __restrict__ hdrs, const DevOp* __restrict__ ops, const T* __restrict__ coef, int pass)
{
    using V = typename CxT<T>::V;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* lds = reinterpret_cast<V*>(smem_raw);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const BatchItem it = items[i];
        const BatchCirc c = circs[it.c];
        const PassHdr* __restrict__ hp = hdrs + c.hdr0 + pass;
        V* __restrict__ st = reinterpret_cast<V*>(c.state);
        const int L = hp->L, nup = hp->nup;
        const uint32_t N = 1u << L;
        const uint64_t base = tile_base((uint64_t)it.tile, hp);
        // the pass's staged coefficients (diagonal tables, matrix-core
        // fragments) follow the tile in LDS, as in the single-circuit kernel
        T* lcoef = reinterpret_cast<T*>(smem_raw + (size_t)N * sizeof(V));
        for (int j = tid; j < hp->coef_n; j += 256) lcoef[j] = coef[hp->coef_src + j];
        for (uint32_t e = tid; e < N; e += 256) {
            V v;
            if (pass == 0) {
                v.x = (base == 0 && e == 0) ? (T)1 : (T)0;
                v.y = 0;
            } else {
                v = st[base + (e & ((1u << QOPS_LDS_FIXED_BITS) - 1u)) + dep_up(e >> QOPS_LDS_FIXED_BITS, hp->up_phys, nup)];
            }
            lds[swz(e)] = v;
        }
        __syncthreads();
        const DevOp* __restrict__ prog = ops + hp->op0;
        for (int j = 0; j < hp->nops; ++j) {
            const DevOp op = prog[j];
            if ((base & op.c_glob) != op.c_glob) continue;
            // ops whose coefficients did not fit next to the tile (op.b = 0;
            // in complex64 the block a single-circuit pass would keep in
            // registers) read them from global memory
            const T* cf = op.b ? lcoef + op.coef : coef + op.coef;
            if (op.type == OP_DENSE_LDS) dense_lds_dispatch<T>(lds, L, op, cf, tid, 256);
            else if (op.type == OP_MFMA) mfma_dispatch<T, 6, 2, 1>(lds, L, op, cf, lane, wave);
            else if (op.type == OP_DIAG_LDS) diag_lds<T>(lds, L, op, cf, base, tid, 256);
            __syncthreads();
        }
        for (uint32_t e = tid; e < N; e += 256) st[base + (e & ((1u << QOPS_LDS_FIXED_BITS) - 1u)) + dep_up(e >> QOPS_LDS_FIXED_BITS, hp->up_phys, nup)] = lds[swz(e)];
        __syncthreads();
    }
}

// <Z> partial sums of the tile-pass circuits: item = (circuit, chunk of
// 2^s amplitudes, s = min(n, 13)); record (n+1 of QOPS_BATCH_REC doubles):
// sum p, sum p bit_q.
template <typename T>
__global__ void __launch_bounds__(256)
batch_zpart_kernel(const BatchItem* __restrict__ items, int nitems, const BatchCirc* __restrict__ circs,
                   double* __restrict__ part)
{
    using V = typename CxT<T>::V;
    __shared__ double sh[256];
    const int t = threadIdx.x;
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const BatchItem it = items[i];
        const BatchCirc c = circs[it.c];
        const int n = c.n, s = n < 13 ? n : 13;
        const V* __restrict__ st = reinterpret_cast<const V*>(c.state);
        const uint64_t base = (uint64_t)it.tile << s;
        double tot = 0.0, sb[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) sb[q] = 0.0;
        for (uint32_t j = 0; (j << 8) < (1u << s); ++j) {
            const uint32_t off = (j << 8) + t;
            if (off >= (1u << s)) break;
            double p;
            if (c.npass == 0) {
                p = (base + off == 0) ? 1.0 : 0.0;     // no gates: still |0..0>
            } else {
                const V v = st[base + off];
                p = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            }
            tot += p;
#pragma unroll
            for (int q = 0; q < 5; ++q)
                if ((j >> q) & 1u) sb[q] += p;
        }
        double* rec = part + (size_t)(c.part0 + it.tile) * QOPS_BATCH_REC;
        const double all = bsum(tot, sh);
        if (t == 0) rec[0] = all;
        for (int q = 0; q < n; ++q) {
            double v;
            if (q < 8 && q < s) {
                v = bsum(((t >> q) & 1) ? tot : 0.0, sh);
            } else if (q < s) {
                double mine = 0.0;
#pragma unroll
                for (int r = 0; r < 5; ++r)
                    if (r == q - 8) mine = sb[r];
                v = bsum(mine, sh);
            } else {
                v = ((base >> q) & 1ull) ? all : 0.0;
            }
            if (t == 0) rec[1 + q] = v;
        }
    }
}

// One work-group per tile-pass circuit: <Z_q> from its partial records, in
// chunk order.
__global__ void __launch_bounds__(256)
batch_zfinal_kernel(const int32_t* __restrict__ ids, const BatchCirc* __restrict__ circs,
                    const double* __restrict__ part, double* __restrict__ out)
{
    __shared__ double sh[256];
    const BatchCirc c = circs[ids[blockIdx.x]];
    const int n = c.n, s = n < 13 ? n : 13;
    const int nch = 1 << (n - s);
    double tot = 0.0;
    for (int k = threadIdx.x; k < nch; k += 256) tot += part[(size_t)(c.part0 + k) * QOPS_BATCH_REC];
    const double all = bsum(tot, sh);
    for (int q = 0; q < n; ++q) {
        double v = 0.0;
        for (int k = threadIdx.x; k < nch; k += 256) v += part[(size_t)(c.part0 + k) * QOPS_BATCH_REC + 1 + q];
        const double sq = bsum(v, sh);
        if (threadIdx.x == 0) out[c.out0 + q] = all - 2.0 * sq;
    }
}

hipError_t launch_batch_small(int prec, const int32_t* ids, int count, const BatchCirc* circs, const DevOp* ops,
                              const void* coef, double* out, int lds_bytes, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (prec == 0) {
        if (hipError_t e = hipFuncSetAttribute((const void*)batch_small_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               lds_bytes))
            return e;
        hipLaunchKernelGGL(batch_small_kernel<float>, dim3(count), dim3(256), lds_bytes, s, ids, circs, ops,
                           reinterpret_cast<const float*>(coef), out);
    } else {
        if (hipError_t e = hipFuncSetAttribute((const void*)batch_small_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               lds_bytes))
            return e;
        hipLaunchKernelGGL(batch_small_kernel<double>, dim3(count), dim3(256), lds_bytes, s, ids, circs, ops,
                           reinterpret_cast<const double*>(coef), out);
    }
    return hipGetLastError();
}

hipError_t launch_batch_pass(int prec, const BatchItem* items, int nitems, const BatchCirc* circs, const PassHdr* hdrs,
                             const DevOp* ops, const void* coef, int pass, int lds_bytes, int grid, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const int g = std::max(1, std::min(nitems, grid));
    if (prec == 0) {
        if (hipError_t e = hipFuncSetAttribute((const void*)batch_pass_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               lds_bytes))
            return e;
        hipLaunchKernelGGL(batch_pass_kernel<float>, dim3(g), dim3(256), lds_bytes, s, items, nitems, circs, hdrs, ops,
                           reinterpret_cast<const float*>(coef), pass);
    } else {
        if (hipError_t e = hipFuncSetAttribute((const void*)batch_pass_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               lds_bytes))
            return e;
        hipLaunchKernelGGL(batch_pass_kernel<double>, dim3(g), dim3(256), lds_bytes, s, items, nitems, circs, hdrs, ops,
                           reinterpret_cast<const double*>(coef), pass);
    }
    return hipGetLastError();
}

template <typename T, int R, int W>
static hipError_t launch_batch_reg_t(const BatchItem* items, int nitems, const BatchCirc* circs, const PassHdr* hdrs,
                                     const DevOp* ops, const void* coef, int pass, int lds_bytes, int grid,
                                     hipStream_t s)
{
    if (hipError_t e = hipFuncSetAttribute((const void*)batch_reg_kernel<T, R, W>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes))
        return e;
    const int g = std::max(1, std::min(nitems, grid));
    hipLaunchKernelGGL((batch_reg_kernel<T, R, W>), dim3(g), dim3(64 << W), lds_bytes, s, items, nitems, circs, hdrs,
                       ops, reinterpret_cast<const T*>(coef), pass);
    return hipGetLastError();
}

hipError_t launch_batch_reg(int prec, int R, int W, const BatchItem* items, int nitems, const BatchCirc* circs,
                            const PassHdr* hdrs, const DevOp* ops, const void* coef, int pass, int lds_bytes,
                            int grid, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
#define QOPS_LAUNCH(r, w)                                                                                      \
    if (R == r && W == w)                                                                                      \
        return prec == 0 ? launch_batch_reg_t<float, r, w>(items, nitems, circs, hdrs, ops, coef, pass, lds_bytes,  \
                                                           grid, s)                                           \
                         : launch_batch_reg_t<double, r, w>(items, nitems, circs, hdrs, ops, coef, pass, lds_bytes, \
                                                            grid, s);
    QOPS_TILE_VARIANTS(QOPS_LAUNCH)
#undef QOPS_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_batch_z(int prec, const BatchItem* items, int nitems, const int32_t* ids, int count,
                          const BatchCirc* circs, double* part, double* out, int grid, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const int g = std::max(1, std::min(nitems, grid));
    if (prec == 0)
        hipLaunchKernelGGL(batch_zpart_kernel<float>, dim3(g), dim3(256), 0, s, items, nitems, circs, part);
    else
        hipLaunchKernelGGL(batch_zpart_kernel<double>, dim3(g), dim3(256), 0, s, items, nitems, circs, part);
    hipLaunchKernelGGL(batch_zfinal_kernel, dim3(count), dim3(256), 0, s, ids, circs, part, out);
    return hipGetLastError();
}

int device_cus() { return num_cus(); }

}  // namespace qops
