// Pass plan: the host-built program that the tiled-pass kernel interprets.
//
// A circuit is cut into passes. A pass owns a set Q of k qubits (the tile
// qubits; always including the lowest few so that HBM accesses are contiguous
// runs) and a list of operations. One workgroup handles one tile: the 2^k
// amplitudes whose non-Q index bits are fixed to the tile's value. It reads
// the tile once, applies every operation of the pass, and writes it back once.
//
// Inside the workgroup a tile is held in registers: thread t (of 2^w) holds
// 2^R amplitudes in register slots j. A "layout" maps (thread bit s, register
// bit p) to tile-local index bits ("labels"), plus an XOR mask c on the labels:
// the amplitude in (t, j) has tile-local index  L(t, j) ^ c. Permutation gates
// on tile qubits are applied by changing the layout instead of moving data
// (SWAP exchanges two labels, X flips a label's XOR bit): the index part of a
// value+index (DAX) entry is absorbed into the addressing, only values remain.
// An EXCH operation re-distributes the tile through LDS into a new layout.
#pragma once

#include <cstddef>
#include <cstdint>

namespace sv {

// Bit sources: where the value of one index bit comes from, for the amplitude a
// thread holds in register slot j (already corrected for the layout's XOR mask
// by the planner, which permutes the operation's constants instead).
enum : uint8_t {
    SRC_REG = 0 << 6,   // bit p of the register slot j (p < R)
    SRC_THR = 1 << 6,   // bit s of the thread index
    SRC_TILE = 2 << 6,  // bit q of the tile's base index (a qubit outside the tile)
    SRC_POS_MASK = 63
};

enum OpCode : uint8_t {
    OP_EXCH = 1,     // write the tile to LDS in layout a, read it back in layout b
                     // (pass-relative), in two halves through a half-tile buffer: the
                     // half is the value of label sb, held at the same position (source
                     // sa: SRC_REG | p or SRC_THR | s) with the same XOR bit in both
                     // layouts; slots drop bit sb
    OP_D1R = 2,      // amp *= f d[bit p of j], f = 1; a = p; payload d0, d1
    OP_UDN = 3,      // per-thread factor f *= C * prod_{i < a} (term i holds ? r_i : 1);
                     // term i is the bit of source s1, or the AND of sources s1 and s2
                     // (s2 != 0xFF); (s1, s2) of terms 0..3 in the bytes of `data`,
                     // of term 4 in (sa, sb); payload C, r_0 .. r_{a-1}
    OP_APPLYF = 5,   // amp *= f for every slot; f = 1
    // 4, 6 and 7: not used
    OP_DENSE1 = 8,   // a 2x2 on register bit a; payload g00 g01 g10 g11; with b = 1 the
                     // matrix is first multiplied by f, and f = 1 (b = 0: f untouched)
    OP_H = 9,        // unscaled Hadamard butterflies (x0 + x1, x0 - x1) on every register
                     // bit set in mask a
    OP_X = 10,       // swap the pairs of register bit a
    OP_CXR = 11,     // swap the pairs of register bit a where register bit b is 1
    OP_CXU = 12,     // swap the pairs of register bit a when the bit of source sa is 1
    OP_MARK = 13,    // amp(slot a, thread sa | sb << 8) *= -1 in the tile whose base equals `data`
    OP_SCALE = 14,   // amp *= s; payload s (one real)
    OP_CXT = 15,     // swap the pairs of register bit a when tile-base bit `sa` (a qubit
                     // outside the tile, the same for the whole workgroup) is 1
    OP_D1H = 16,     // amp *= d for the slots whose register bit a equals b (f untouched)
    OP_D2Q = 17,     // amp *= d for the slots whose register bits a, b equal bits 0, 1 of sa
    OP_D1HU = 18,    // amp *= d for the slots whose register bit a equals bit 0 of b, when
                     // the bit of source sa equals bit 1 of b (f untouched)
    OP_RPERM = 19,   // exchange register bits a and b (slots j with bit a = 1, bit b = 0
                     // swap with j ^ 2^a ^ 2^b)
    OP_DENSE2 = 20,  // 4x4 on register bits 1 (high) and 0 (low): entries row-major, the
                     // first ones in this payload, the rest in the OP_CONT records after it
    OP_CONT = 21,    // continuation of the preceding operation's payload (not executed)
    OP_DENSE1RI = 22,  // a 2x2 whose entries are each real or imaginary, on register bit a:
                       // diag(i^g0, i^g1) R diag(1, i^bt) with R real (payload r00 r01 r10
                       // r11), g0 = bit 0 of b, g1 = bit 1, bt = bit 2 (f untouched)
    OP_CCX = 23,       // swap the pairs of register bit a in the slots j with
                       // (j & b) == data byte 0 (register controls), in the threads where
                       // the bits of sources sa, sb (0xFF: none) equal bits 0, 1 of data byte 1
    OP_GENP = 24,      // product-state generation data of a PASS_GEN_PRODUCT pass (its first
                       // record; not executed): for qubit q, u_q = (u_q0, u_q1) complex FP64
                       // (both precisions) in record q / 2 at entries 4 (q % 2) .. + 3,
                       // continued in the b OP_CONT records after it; a = n
};

constexpr uint8_t kNoSource = 0xFF;
constexpr int kMaxUdTerms = 5;       // OP_UDN terms (term descriptors in the header)
constexpr int kMaxUdTermsC128 = 3;   // complex128: C and 3 ratios fill the payload

// One operation: 16-byte header and 64-byte payload (8 doubles or 16 floats:
// the constants in the precision of the state). Stored per batch entry.
struct DevOp {
    uint8_t code;
    uint8_t a;
    uint8_t b;
    uint8_t sa;
    uint8_t sb;
    uint8_t pad[3];
    uint64_t data;
    uint64_t payload[8];
};

// Largest tile geometry the plan records describe.
constexpr int kLayoutThreadBits = 10;
constexpr int kLayoutRegBits = 6;

// Per-layout tables, precomputed on the host. The global index of the
// amplitude in (t, j) is  tile_base | gthr(t) | greg(j)  (disjoint bits) with
//   gthr(t) = goff_xor ^ XOR_{s: t_s = 1} thr_goff[s],
//   greg(j) = reg_goff_xor ^ XOR_{p: j_p = 1} reg_goff[p],
// and its LDS slot (swizzled) is  sthr(t) ^ sreg(j), built the same way.
// Entries of thread bits at or above the workgroup's width are zero.
struct DevLayout {                           // 256 bytes
    uint64_t thr_goff[kLayoutThreadBits];
    uint64_t reg_goff[kLayoutRegBits];
    uint64_t goff_xor;       // global offset of the XOR-mask labels held by thread bits
    uint64_t reg_goff_xor;   // global offset of the XOR-mask labels held by register bits
    uint32_t thr_slot[kLayoutThreadBits];
    uint32_t reg_slot[kLayoutRegBits];
    uint32_t slot_xor;       // LDS slot contribution of the whole XOR mask
    uint32_t flags;          // LAYOUT_PAIR_IO: slots j, j^1 are adjacent in HBM (complex64 16-byte I/O)
    uint32_t xor_local;      // XOR mask c on the labels
    uint8_t thr_local[kLayoutThreadBits];    // label held by thread bit s
    uint8_t reg_local[kLayoutRegBits];       // label held by register bit p
    uint8_t pad[20];
};

enum : uint32_t { LAYOUT_PAIR_IO = 1u };

enum : uint32_t {
    PASS_GENERATE = 1u,     // no load: amplitudes of H^M |j> generated in place
    PASS_SYNC_STORE = 2u,   // barrier before the store: the store layout moves amplitudes
                            // between waves and no exchange has separated loads from stores
    PASS_DENSE2 = 4u,       // the pass holds OP_DENSE2 (run by the kernel variant with it)
    PASS_GEN_PRODUCT = 8u,  // no load: the product state amp[i] = prod_q u_q[bit q of i]
                            // generated in place (u from the pass's OP_GENP records)
    PASS_GENERATES = PASS_GENERATE | PASS_GEN_PRODUCT,   // the pass reads nothing
};

struct DevPass {      // 96 bytes
    int32_t k;              // tile qubits
    int32_t w;              // thread bits (2^w threads; k = w + R)
    int32_t op_begin;       // index into the op array of a batch entry
    int32_t op_end;
    int32_t layout_begin;   // index of this pass's layout 0 (the load layout)
    uint32_t flags;
    uint64_t tiles;         // 2^(n - k)
    uint64_t gen_j;         // generation: basis state j
    uint64_t gen_mask;      // generation: Hadamard qubit mask M
    double gen_scale;       // generation: magnitude 2^(-|M|/2) times folded scale
    int32_t store_layout;   // pass-relative index of the layout the tile is stored from
    uint8_t q[28];          // global qubit of tile-local bit l (ascending)
    int32_t n_layouts;      // layouts of this pass: [layout_begin, layout_begin + n_layouts)
    uint8_t pad[4];
};

static_assert(sizeof(DevOp) == 80, "DevOp layout");
static_assert(sizeof(DevLayout) == 256, "DevLayout layout");
static_assert(sizeof(DevPass) == 96, "DevPass layout");
static_assert(offsetof(DevPass, q) % 4 == 0, "DevPass::q is read as 32-bit words");

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
    SOP_CCX = 11,     // q0, q1 = controls, q2 = target
};

struct SmallOp {      // 16 bytes
    uint8_t code;
    uint8_t q0;
    uint8_t q1;
    uint8_t q2;       // SOP_CCX: target
    uint8_t pad[4];
    uint64_t data;
};
static_assert(sizeof(SmallOp) == 16, "SmallOp layout");

// One request of a heterogeneous small-state group (serving): the workgroup
// with this index builds |0...0> in LDS, runs n_ops small ops starting at
// op_begin with constants at const_begin (reals), and writes <Z_qubit>.
struct SmallJob {     // 32 bytes
    int32_t n;
    int32_t qubit;
    int32_t op_begin;
    int32_t n_ops;
    uint64_t const_begin;
    uint64_t pad;
};
static_assert(sizeof(SmallJob) == 32, "SmallJob layout");

// Continuous batching of tiled states: one launch advances every request
// of a step by one pass of its own plan. StepReq: a request's state, the byte
// offsets of its plan records in the engine's plan arena (passes and layouts
// of its circuit, its own op records) and the pass this step runs; StepItem:
// one workgroup's request (index into the step's StepReq table) and tile.
struct StepReq {      // 48 bytes
    void *state;
    uint64_t passes_off;
    uint64_t layouts_off;
    uint64_t ops_off;
    int32_t pass;
    int32_t n;
    uint64_t pad;
};
static_assert(sizeof(StepReq) == 48, "StepReq layout");
struct StepItem {     // 8 bytes
    uint32_t req;
    uint32_t tile;
};
static_assert(sizeof(StepItem) == 8, "StepItem layout");

// Readout of several states in one launch: work item b sums the amplitudes
// [blk * chunk, (blk + 1) * chunk) of `state` with the signs of <Z_qubit>
// into partial `part` (the same order as the single-state reduction).
struct RedItem {      // 32 bytes
    const void *state;
    uint64_t chunk;
    uint32_t blk;
    int32_t qubit;
    uint32_t part;
    uint32_t pad;
};
static_assert(sizeof(RedItem) == 32, "RedItem layout");
// Final sums: out[slot] = the fixed-tree sum of partials [first, first + count).
struct FinItem {      // 16 bytes
    uint32_t first;
    uint32_t count;
    uint32_t slot;
    uint32_t pad;
};
static_assert(sizeof(FinItem) == 16, "FinItem layout");

}  // namespace sv
