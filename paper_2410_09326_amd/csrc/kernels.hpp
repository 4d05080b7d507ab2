// Launch functions of the simulator kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "devprog.hpp"

namespace qops {

// Tile kernel variants (register bits R, wave bits W): tile bits L = 6+R+W.
struct TileVariant {
    int R, W;
};
bool tile_variant_supported(int prec, int R, int W);
int tile_max_lds_bytes();

// One fused tile pass.  `hdr`, `ops`, `coef` are device pointers; `lds_bytes`
// is the dynamic LDS the pass needs (0 when it has no LDS op).
hipError_t launch_tile_pass(int prec, int R, int W, void* state, const PassHdr* hdr, const DevOp* ops,
                            const void* coef, uint64_t ntiles, int lds_bytes, int grid_cap, hipStream_t s);

// LDS tile pass (dense blocks): tile of 2^L amplitudes in LDS, 256 threads,
// in one static LDS block per work-group (80 KiB complex64, 160 KiB
// complex128); `lds_bytes` (tile plus staged coefficients) must fit in it,
// else hipErrorInvalidValue.  hoist_k: qubits of the block whose fragments
// stay in registers (hdr->hoist), 0 if none.
hipError_t launch_tile_lds(int prec, void* state, const PassHdr* hdr, const DevOp* ops, const void* coef,
                           uint64_t ntiles, int L, int lds_bytes, int grid_cap, int hoist_k, hipStream_t s);

// Whole state in one work-group's LDS (n <= 13 for c64, <= 12 for c128).
hipError_t launch_state_lds(int prec, void* state, int n, const DevOp* ops, int nops, const void* coef,
                            hipStream_t s);

// Gate-wise HBM sweep of one operation (types OP_DENSE_LDS / OP_DIAG_LDS
// with physical bit positions; "tile" = whole state).  grid_cap > 0 limits
// the work-groups; the kernel walks the rest in a grid-stride loop.
hipError_t launch_sweep(int prec, void* state, int n, const DevOp* op_host, const void* coef_dev, int grid_cap,
                        hipStream_t s);

// Exchange of physical bits a and b (a != b); grid_cap as for launch_sweep.
hipError_t launch_swap_bits(int prec, void* state, int n, int a, int b, int grid_cap, hipStream_t s);

// Writes |x>: zero everywhere, one at x.
hipError_t launch_init_basis(int prec, void* state, int n, uint64_t x, hipStream_t s);

// FP64 reductions.  zsum: out[0] = sum p, out[1+b] = sum p*bit_b(x) for
// every physical bit b (n+1 doubles, device pointer); `scratch` must hold
// zsum_scratch_doubles(n) doubles.
size_t zsum_scratch_doubles(int n);
hipError_t launch_zsum(int prec, const void* state, int n, double* scratch, double* out, hipStream_t s);
// <Z_q> of every logical qubit q (l2p: host array of n entries) into out
// (n doubles, device).  The partial records are bounded: `scratch` must hold
// zsum_bounded_scratch_doubles(n) doubles, at most 2^11 * 35 + 35 for n <= 34.
struct ZLayout {
    int32_t l2p[QOPS_MAX_QUBITS_DEV];
};
size_t zsum_bounded_scratch_doubles(int n);
hipError_t launch_expect_z_bounded(int prec, const void* state, int n, const int32_t* l2p, double* scratch,
                                   double* out, hipStream_t s);

// Marginal over physical bits pos[0..m-1] (host array); out: 2^m doubles
// (device).  scratch must hold probs_scratch_doubles(n, m, pos) doubles.
size_t probs_scratch_doubles(int n, int m, const int* pos);
hipError_t launch_probs(int prec, const void* state, int n, int m, const int* pos, double* scratch,
                        double* out, hipStream_t s);

// Gathers logical-order amplitudes [x0, x0+count) into dst (device):
// dst[i] = state[phys(x0+i)], phys(x) = sum_q b_q(x) << l2p[q].
hipError_t launch_gather_logical(int prec, const void* state, int n, const int* l2p, uint64_t x0,
                                 uint64_t count, void* dst, hipStream_t s);

// Batched executor kernels.
#define QOPS_BATCH_SMALL_MAX 13
#define QOPS_BATCH_REC 32   // doubles per <Z> partial record (n + 1 <= 27)
// <Z_a Z_b> for physical bit pairs (pa[i], pb[i]): partials in `part`
// (zz_scratch_doubles(n) doubles), results in d_out[0..npairs).
size_t zz_scratch_doubles(int n);
hipError_t launch_expect_zz(int prec, const void* state, int n, const int32_t* pa, const int32_t* pb, int npairs,
                            double* part, double* d_out, hipStream_t s);

hipError_t launch_batch_small(int prec, const int32_t* ids, int count, const BatchCirc* circs, const DevOp* ops,
                              const void* coef, double* out, int lds_bytes, hipStream_t s);
hipError_t launch_batch_pass(int prec, const BatchItem* items, int nitems, const BatchCirc* circs, const PassHdr* hdrs,
                             const DevOp* ops, const void* coef, int pass, int lds_bytes, int grid, hipStream_t s);
// Batched register-tile pass `pass` over (circuit, tile) items of one R/W split.
hipError_t launch_batch_reg(int prec, int R, int W, const BatchItem* items, int nitems, const BatchCirc* circs,
                            const PassHdr* hdrs, const DevOp* ops, const void* coef, int pass, int lds_bytes,
                            int grid, hipStream_t s);
hipError_t launch_batch_z(int prec, const BatchItem* items, int nitems, const int32_t* ids, int count,
                          const BatchCirc* circs, double* part, double* out, int grid, hipStream_t s);
int device_cus();

}  // namespace qops
