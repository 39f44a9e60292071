// Pass plan: the host-built program that the tiled-pass kernel interprets.
//
// A circuit is cut into passes. A pass owns a set Q of k qubits (the tile
// qubits; always including the lowest few so that HBM accesses are contiguous
// runs) and a list of operations. One workgroup handles one tile: the 2^k
// amplitudes whose non-Q index bits are fixed to the tile's value. It reads
// the tile once, applies every operation of the pass, and writes it back once.
//
// Inside the workgroup a tile is held in registers: thread t (of 2^w) holds
// 2^R amplitudes. A "layout" says which tile-local bits are register bits and
// which are thread bits. Gates whose non-diagonal part lives on register bits
// are applied without communication; an EXCH operation re-distributes the tile
// through LDS into a new layout. Diagonal gates need no register bits at all:
// each thread knows the global index of every amplitude it holds.
#pragma once

#include <cstdint>

namespace sv {

// Bit sources: where the value of one global index bit comes from, for the
// amplitude a thread holds in register slot j.
enum : uint8_t {
    SRC_REG = 0 << 6,   // bit p of the register slot j (p < R)
    SRC_THR = 1 << 6,   // bit s of the thread index
    SRC_TILE = 2 << 6,  // bit q of the tile's base index (outside the tile)
    SRC_POS_MASK = 63
};

enum OpCode : uint8_t {
    OP_EXCH = 1,     // a = layout index within the pass
    OP_D1 = 2,       // 1-qubit diagonal: amp *= d[bit];   sa; data = const offset (4 reals)
    OP_D2 = 3,       // 2-qubit diagonal: amp *= d[(b0<<1)|b1]; sa, sb; data (8 reals)
    OP_MARK = 4,     // amp[idx == m] *= -1: a = register slot, b = thread, data = tile base of m
    OP_DENSE1 = 5,   // 2x2 on register bit a; data (8 reals, row-major g00 g01 g10 g11)
    OP_H = 6,        // unscaled Hadamard butterfly (x0 + x1, x0 - x1) on register bit a
    OP_X = 7,        // swap pairs on register bit a
    OP_Y = 8,        // (x0, x1) -> (-i x1, i x0) on register bit a
    OP_CX = 9,       // controlled swap on register bit a, control bit source sa
    OP_SWAP = 10,    // swap of register bits a, b (a > b)
    OP_DENSE2 = 11,  // 4x4 on register bits a (high local bit) and b (low), a > b; data (32 reals)
    OP_SCALE = 12,   // amp *= s (real); data (1 real)
};

struct DevOp {        // 16 bytes
    uint8_t code;
    uint8_t a;
    uint8_t b;
    uint8_t sa;
    uint8_t sb;
    uint8_t pad[3];
    uint64_t data;
};

struct DevLayout {    // 16 bytes
    uint8_t reg_local[8];   // tile-local bit held by register bit p
    uint8_t thr_local[8];   // tile-local bit held by thread bit s
};

enum : uint32_t {
    PASS_GENERATE = 1u,     // no load: amplitudes of H^M |j> generated in place
};

struct DevPass {      // 96 bytes
    int32_t k;              // tile qubits
    int32_t w;              // thread bits (2^w threads; k = w + R)
    int32_t op_begin;       // index into the op array
    int32_t op_end;
    int32_t layout_begin;   // index of this pass's layout 0 (the load layout)
    uint32_t flags;
    uint64_t tiles;         // 2^(n - k)
    uint64_t gen_j;         // generation: basis state j
    uint64_t gen_mask;      // generation: Hadamard qubit mask M
    double gen_scale;       // generation: magnitude 2^(-|M|/2) times folded scale
    uint8_t q[32];          // global qubit of tile-local bit l (ascending)
    uint8_t pad[8];
};

static_assert(sizeof(DevOp) == 16, "DevOp layout");
static_assert(sizeof(DevLayout) == 16, "DevLayout layout");
static_assert(sizeof(DevPass) == 96, "DevPass layout");

// Ops of the one-workgroup small-state kernel: the whole state sits in LDS.
enum SmallCode : uint8_t {
    SOP_D1 = 1,       // q0; data = const offset (4 reals)
    SOP_D2 = 2,       // q0 (high), q1; data (8 reals)
    SOP_MARK = 3,     // data = basis index
    SOP_DENSE1 = 4,   // q0; data (8 reals)
    SOP_DENSE2 = 5,   // q0, q1; data (32 reals)
    SOP_X = 6,        // q0
    SOP_Y = 7,        // q0
    SOP_CX = 8,       // q0 = control, q1 = target
    SOP_SWAP = 9,     // q0, q1
    SOP_SCALE = 10,   // data (1 real)
};

struct SmallOp {      // 16 bytes
    uint8_t code;
    uint8_t q0;
    uint8_t q1;
    uint8_t pad[5];
    uint64_t data;
};
static_assert(sizeof(SmallOp) == 16, "SmallOp layout");

}  // namespace sv
