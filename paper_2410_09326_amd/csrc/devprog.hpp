// Device-side pass programs: the plain-old-data records the planner writes
// and the kernels read.  Shared between host (planner/runtime) and device
// (kernels) translation units of libqops.
#pragma once
#include <stdint.h>

namespace qops {

// Operation types inside a tile pass.
enum OpType : int32_t {
    OP_NONE = 0,
    OP_1Q_REG = 1,    // 2x2 on a register bit          a = register bit
    OP_1Q_LANE = 2,   // 2x2 on a lane bit (shuffles)    a = lane bit (0..5)
    OP_DIAG = 3,      // diagonal table over m bits      a = m, pos[i] = encoded source of bit i
    OP_REMAP = 4,     // registers -> LDS -> registers   b = new mapping
    OP_TO_LDS = 5,    // registers -> LDS
    OP_FROM_LDS = 6,  // LDS -> registers                b = new mapping
    OP_DENSE_LDS = 7, // 2^k x 2^k on tile positions, vector ALU, in LDS   a = k, pos = tile positions
    OP_MFMA = 8,      // 2^k x 2^k on tile positions, matrix cores, in LDS  a = k, pos = tile positions
    OP_DIAG_LDS = 9,  // diagonal table on tile positions, in LDS (whole-state kernel)
    OP_CPHASE = 10    // phase coef on amplitudes whose masked bits are all 1   b = 1: phase is -1
};
// OP_1Q_REG / OP_1Q_LANE: b = 1 marks an exact X (pure exchange, no arithmetic).
// OP_MFMA / OP_DIAG_LDS / OP_DENSE_LDS in an LDS tile pass: b = 1 means `coef` is an offset
// into the coefficients staged in LDS, b = 0 an offset into global memory.
// OP_MFMA: c_reg (unused by LDS ops otherwise) holds QOPS_MFMA_WIDE when the
// block runs in the 32x32x2 three-product form (5-qubit blocks on the
// largest complex64 tile); its coefficients then follow that layout.
#define QOPS_MFMA_WIDE 1u

// Encoded source of one bit of a diagonal's table index (OP_DIAG pos[i]).
enum BitSrc : int32_t { SRC_LANE = 0, SRC_WAVE = 1, SRC_REG = 2, SRC_GLOB = 3 };
__host__ __device__ inline int32_t enc_src(int32_t cls, int32_t v) { return (cls << 8) | v; }

struct DevOp {              // 64 bytes
    int32_t type;
    int32_t a;
    int32_t coef;           // offset of the coefficients in the coefficient array (scalar units)
    int32_t b;
    uint32_t c_lane;        // controls on lane bits (tile positions 0..5)
    uint32_t c_wave;        // controls on wave-id bits (current mapping)
    uint32_t c_reg;         // controls on register-slot bits (current mapping)
    uint32_t c_tile;        // controls on tile positions (LDS ops)
    uint64_t c_glob;        // controls on physical bits outside the tile (checked per tile)
    int32_t pos[6];
};
static_assert(sizeof(DevOp) == 64, "DevOp layout");

#define QOPS_MAX_UP 10
// LDS tile passes hold physical bits 0..3 contiguously (128-byte runs of
// complex64) and choose every other tile bit; register tile passes hold bits
// 0..5 in the lanes of a wave.
#define QOPS_LDS_FIXED_BITS 4
// LDS of one work-group of the LDS tile kernel (tile plus staged
// coefficients): complex64 runs two work-groups per CU, complex128 one.
#define QOPS_LDS_TILE_BYTES_C64 (80 * 1024)
#define QOPS_LDS_TILE_BYTES_C128 (160 * 1024)
#define QOPS_MAX_QUBITS_DEV 34
#define QOPS_MAX_RUNS 12

// Header of one tile pass.  The tile holds 2^L amplitudes: tile positions
// 0..F-1 are physical bits 0..F-1 and tile position F+u is physical bit
// up_phys[u], with F = 6 for register tile passes (one lane bit each) and
// F = QOPS_LDS_FIXED_BITS for LDS tile passes.  The other physical bits
// index the tile.
struct PassHdr {
    int32_t n;
    int32_t L;
    int32_t nup;                    // L - F
    int32_t nops;
    int32_t op0;                    // first op in the op array
    uint32_t map0;                  // mapping used for the load
    int32_t nruns;                  // runs of non-tile physical bits
    int32_t lds_bytes;              // LDS the pass needs (0 if no LDS op)
    int32_t coef_src;               // LDS tile pass: coefficients staged into LDS once per
    int32_t coef_n;                 //   work-group: coef[coef_src .. coef_src + coef_n)
    int32_t up_phys[QOPS_MAX_UP];
    int32_t run_start[QOPS_MAX_RUNS];  // physical start bit of each run
    int32_t run_len[QOPS_MAX_RUNS];
    int32_t run_gshift[QOPS_MAX_RUNS]; // bit offset of the run inside the tile number
    int32_t hoist;                  // LDS tile pass: op (relative to op0) whose matrix-core
                                    //   fragments stay in registers, or -1
};

// Batched executor records.
struct BatchCirc {
    void* state;        // circuits run in tile passes: their state buffer
    int32_t n;
    int32_t npass;      // tile passes
    int32_t hdr0;       // first pass header in the batch's header array
    int32_t out0;       // offset of the circuit's n <Z> outputs
    int32_t op0;        // whole-state circuits: their operations
    int32_t nops;
    int32_t part0;      // first partial-sum record of the <Z> reduction
    int32_t pad;
};
struct BatchItem {
    int32_t c;          // circuit
    int32_t tile;       // tile (pass kernels) or chunk (reduction)
};

// A mapping assigns the upper tile positions to register bits (first R
// nibbles) and wave bits (next W nibbles).
__host__ __device__ inline int32_t map_get(uint32_t m, int i) { return (int32_t)((m >> (4 * i)) & 15u); }

}  // namespace qops
