// gfx950 kernels of the state-vector engine.
//
// k_pass   — one fused pass over HBM: a workgroup loads a tile of 2^k
//            amplitudes into registers, runs the pass's operation list
//            (gates on register bits without communication, diagonal gates on
//            any qubit from the global index, re-layouts through LDS), and
//            writes the tile back. This applies U|phi> of the paper's
//            Sec. II-A for a run of gates without forming U; sparse gates are
//            applied from their gate-local (value, index) form in the spirit of
//            DAX (Sec. III-A: only non-zeros are touched), Hadamards as
//            on-demand sign butterflies with one magnitude per pass (RH,
//            Sec. III-B).
// k_small  — the whole state in one workgroup's LDS (small n).
// k_reduce — <Z_q> and norm with FP64 accumulation in a fixed order.
// k_gather — amplitude readout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "sv_kernels.hpp"
#include "sv_plan.hpp"

namespace sv {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T x, T y) {
    cpx<T> r;
    r.x = x;
    r.y = y;
    return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) {
    return mk<T>(a.x + b.x, a.y + b.y);
}
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) {
    return mk<T>(a.x - b.x, a.y - b.y);
}
// a*x + b*y
template <typename T>
__device__ __forceinline__ cpx<T> cmul2(cpx<T> a, cpx<T> x, cpx<T> b, cpx<T> y) {
    return mk<T>(a.x * x.x - a.y * x.y + b.x * y.x - b.y * y.y,
                 a.x * x.y + a.y * x.x + b.x * y.y + b.y * y.x);
}
template <typename T>
__device__ __forceinline__ cpx<T> ldc(const T *p) {
    return mk<T>(p[0], p[1]);
}

// Pass traffic: each amplitude is read once and written once per pass, so
// tile loads and stores carry the non-temporal hint (measured on the device:
// a streaming in-place read-modify-write runs faster with it).
template <typename T>
__device__ __forceinline__ cpx<T> ld_stream(const cpx<T> *p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
    return mk<T>(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void st_stream(cpx<T> *p, cpx<T> a) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, reinterpret_cast<v2 *>(p));
}
// two adjacent complex64 amplitudes as one 16-byte access
__device__ __forceinline__ void ld_stream2(const cpx<float> *p, cpx<float> &a0, cpx<float> &a1) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = __builtin_nontemporal_load(reinterpret_cast<const v4 *>(p));
    a0 = mk<float>(v.x, v.y);
    a1 = mk<float>(v.z, v.w);
}
__device__ __forceinline__ void st_stream2(cpx<float> *p, cpx<float> a0, cpx<float> a1) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    v4 v;
    v.x = a0.x;
    v.y = a0.y;
    v.z = a1.x;
    v.w = a1.y;
    __builtin_nontemporal_store(v, reinterpret_cast<v4 *>(p));
}

// Workgroups go round-robin to the 8 XCDs (workgroup b to XCD b mod 8). Give
// each XCD one contiguous eighth of the tile numbers instead: measured on the
// device, streaming passes over the state run faster that way. A bijection
// on [0, g) when g is a multiple of 8, the identity otherwise.
__device__ __forceinline__ uint64_t xcd_tile(uint32_t b, uint32_t g) {
    return (g & 7u) ? (uint64_t)b : (uint64_t)(b & 7u) * (g >> 3) + (b >> 3);
}

// ---------------------------------------------------------------------------
// Register-tile operations. P, PA, PB are register-bit positions (compile
// time); every loop is fully unrolled so the tile never leaves VGPRs.

// In-place forms: every new value is computed so that it can take the
// register of the old value it replaces (no temporaries live across the
// update), which keeps the register tile in fixed VGPRs across the
// interpreter's dispatch merge.

// a *= d
template <typename T>
__device__ __forceinline__ void cmul_ip(cpx<T> &a, cpx<T> d) {
    a = cmul(a, d);
}

// Exchange two register values without renaming them: each asm output is
// tied to its input VGPR, so a permutation of the register tile is a
// physical exchange and the tile keeps fixed VGPRs across the interpreter's
// dispatch merge (a renamed permutation there costs a whole-tile copy on
// every operation).
__device__ __forceinline__ void vswap32(uint32_t &x, uint32_t &y) {
    asm volatile("v_swap_b32 %0, %1" : "+v"(x), "+v"(y));
}
template <typename T>
__device__ __forceinline__ void vswap(T &x, T &y);
template <>
__device__ __forceinline__ void vswap<double>(double &x, double &y) {
    const uint64_t a = __builtin_bit_cast(uint64_t, x), b = __builtin_bit_cast(uint64_t, y);
    uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32), bl = (uint32_t)b, bh = (uint32_t)(b >> 32);
    vswap32(al, bl);
    vswap32(ah, bh);
    x = __builtin_bit_cast(double, ((uint64_t)ah << 32) | al);
    y = __builtin_bit_cast(double, ((uint64_t)bh << 32) | bl);
}
template <>
__device__ __forceinline__ void vswap<float>(float &x, float &y) {
    uint32_t a = __builtin_bit_cast(uint32_t, x), b = __builtin_bit_cast(uint32_t, y);
    vswap32(a, b);
    x = __builtin_bit_cast(float, a);
    y = __builtin_bit_cast(float, b);
}
template <typename T>
__device__ __forceinline__ void cswap(cpx<T> &p, cpx<T> &q) {
    vswap(p.x, q.x);
    vswap(p.y, q.y);
}

// Toffoli on register bit P: swap the pairs whose slot bits under the
// register-control mask cm equal cv (uniform values: a scalar branch per slot).
template <int P, typename T, int NR>
__device__ __forceinline__ void r_ccx(cpx<T> (&a)[NR], uint32_t cm, uint32_t cv) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        if (((uint32_t)j & cm) == cv) cswap(a[j], a[j | (1 << P)]);
    }
}

// Hadamard butterfly (x0 + x1, x0 - x1) as x0 <- x0 + x1, x1 <- x0' - 2 x1
template <int P, typename T, int NR>
__device__ __forceinline__ void r_h(cpx<T> (&a)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        const int j1 = j | (1 << P);
        a[j].x = a[j].x + a[j1].x;
        a[j1].x = __builtin_fma((T)-2, a[j1].x, a[j].x);
        a[j].y = a[j].y + a[j1].y;
        a[j1].y = __builtin_fma((T)-2, a[j1].y, a[j].y);
    }
}

// The 2x2 diag(i^G0, i^G1) R diag(1, i^BT) on register bit P, R real: two
// real products per complex output instead of four. The factors of i are
// re/im renames and signs, folded into the multiply-adds.
template <int P, int G0, int G1, int BT, typename T, int NR>
__device__ __forceinline__ void r_dense1_ri(cpx<T> (&a)[NR], T r00, T r01, T r10, T r11) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        const int j1 = j | (1 << P);
        const cpx<T> x0 = a[j], x1 = a[j1];
        const T y1r = BT ? -x1.y : x1.x, y1i = BT ? x1.x : x1.y;   // i^BT x1
        const T z0r = r00 * x0.x + r01 * y1r, z1r = r10 * x0.x + r11 * y1r;
        // a factor i on an output: (re, im) <- (-im, re), the sign taken into
        // the products (a negated operand costs no instruction)
        if constexpr (G0) a[j] = mk<T>(-r00 * x0.y - r01 * y1i, z0r);
        else a[j] = mk<T>(z0r, r00 * x0.y + r01 * y1i);
        if constexpr (G1) a[j1] = mk<T>(-r10 * x0.y - r11 * y1i, z1r);
        else a[j1] = mk<T>(z1r, r10 * x0.y + r11 * y1i);
    }
}

template <int P, typename T, int NR>
__device__ __forceinline__ void r_dense1(cpx<T> (&a)[NR], cpx<T> g00, cpx<T> g01, cpx<T> g10,
                                         cpx<T> g11) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        const int j1 = j | (1 << P);
        const cpx<T> x0 = a[j];
        // x1 <- g10 x0 + g11 x1 (last use of x1 is here), then x0 from the copy
        const T nx1 = g10.x * x0.x - g10.y * x0.y + g11.x * a[j1].x - g11.y * a[j1].y;
        const T ny1 = g10.x * x0.y + g10.y * x0.x + g11.x * a[j1].y + g11.y * a[j1].x;
        const T nx0 = g00.x * x0.x - g00.y * x0.y + g01.x * a[j1].x - g01.y * a[j1].y;
        const T ny0 = g00.x * x0.y + g00.y * x0.x + g01.x * a[j1].y + g01.y * a[j1].x;
        a[j1].x = nx1;
        a[j1].y = ny1;
        a[j].x = nx0;
        a[j].y = ny0;
    }
}

template <int P, typename T, int NR>
__device__ __forceinline__ void r_x(cpx<T> (&a)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        cswap(a[j], a[j | (1 << P)]);
    }
}

// Swap the pairs of bit P in the slots whose bit PC is set.
template <int P, int PC, typename T, int NR>
__device__ __forceinline__ void r_cx_reg(cpx<T> (&a)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        if (!(j & (1 << PC))) continue;
        cswap(a[j], a[j | (1 << P)]);
    }
}

// Swap the pairs of bit P when c (the same for every slot of this thread):
// per-component selects, no branch.
template <int P, typename T, int NR>
__device__ __forceinline__ void r_cx_uni(cpx<T> (&a)[NR], bool c) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        const int j1 = j | (1 << P);
        const T x0 = a[j].x, y0 = a[j].y, x1 = a[j1].x, y1 = a[j1].y;
        a[j].x = c ? x1 : x0;
        a[j].y = c ? y1 : y0;
        a[j1].x = c ? x0 : x1;
        a[j1].y = c ? y0 : y1;
    }
}

template <int P, typename T, int NR>
__device__ __forceinline__ void r_d1_reg(cpx<T> (&a)[NR], cpx<T> d0, cpx<T> d1) {
#pragma unroll
    for (int j = 0; j < NR; ++j) cmul_ip(a[j], (j & (1 << P)) ? d1 : d0);
}

// Exchange register bits PA and PB: slots with bit PA set and PB clear swap
// with the slot that has them the other way round.
template <int PA, int PB, typename T, int NR>
__device__ __forceinline__ void r_rperm(cpx<T> (&a)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (((j >> PA) & 1) && !((j >> PB) & 1)) cswap(a[j], a[j ^ (1 << PA) ^ (1 << PB)]);
}

// amp *= d for the slots whose register bit P equals V
template <int P, int V, typename T, int NR>
__device__ __forceinline__ void r_d1_half(cpx<T> (&a)[NR], cpx<T> d) {
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (((j >> P) & 1) == V) cmul_ip(a[j], d);
}

// amp *= d for the slots whose register bit P equals V and whose bit pb
// (uniform, run time) equals xb
template <int P, int V, int PB, int VB, typename T, int NR>
__device__ __forceinline__ void r_d1_quarter(cpx<T> (&a)[NR], cpx<T> d) {
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (((j >> P) & 1) == V && ((j >> PB) & 1) == VB) cmul_ip(a[j], d);
}


template <typename T, int NR>
__device__ __forceinline__ void r_mul_all(cpx<T> (&a)[NR], cpx<T> d) {
#pragma unroll
    for (int j = 0; j < NR; ++j) cmul_ip(a[j], d);
}

template <typename T, int NR>
__device__ __forceinline__ void r_scale(cpx<T> (&a)[NR], T s) {
#pragma unroll
    for (int j = 0; j < NR; ++j) a[j] = mk<T>(a[j].x * s, a[j].y * s);
}

// Dispatch of a runtime register-bit position onto a compile-time one.
#define SV_CASE_A(P, ...)                     \
    case P:                                   \
        if constexpr ((P) < R) {              \
            constexpr int PA = (P);           \
            __VA_ARGS__;                      \
        }                                     \
        break;
#define SV_SWITCH_A(v, ...)                                                    \
    switch (v) {                                                               \
        SV_CASE_A(0, __VA_ARGS__) SV_CASE_A(1, __VA_ARGS__)                    \
        SV_CASE_A(2, __VA_ARGS__) SV_CASE_A(3, __VA_ARGS__)                    \
        SV_CASE_A(4, __VA_ARGS__) SV_CASE_A(5, __VA_ARGS__) default : break;   \
    }
#define SV_CASE_B(P, ...)                     \
    case P:                                   \
        if constexpr ((P) < R) {              \
            constexpr int PB = (P);           \
            __VA_ARGS__;                      \
        }                                     \
        break;
#define SV_SWITCH_B(v, ...)                                                    \
    switch (v) {                                                               \
        SV_CASE_B(0, __VA_ARGS__) SV_CASE_B(1, __VA_ARGS__)                    \
        SV_CASE_B(2, __VA_ARGS__) SV_CASE_B(3, __VA_ARGS__)                    \
        SV_CASE_B(4, __VA_ARGS__) SV_CASE_B(5, __VA_ARGS__) default : break;   \
    }

// An operation record as the kernel reads it: the same 80 bytes as DevOp,
// with the byte fields of the header taken from two aligned 32-bit words
// (a byte field read on its own can become a vector load whose latency the
// interpreter would wait out on every operation).
struct OpRec {
    uint32_t h0;            // code | a << 8 | b << 16 | sa << 24
    uint32_t h1;            // sb | pad
    uint64_t data;
    uint64_t payload[8];
    __device__ __forceinline__ uint32_t code() const { return h0 & 0xFFu; }
    __device__ __forceinline__ uint32_t a() const { return (h0 >> 8) & 0xFFu; }
    __device__ __forceinline__ uint32_t b() const { return (h0 >> 16) & 0xFFu; }
    __device__ __forceinline__ uint32_t sa() const { return h0 >> 24; }
    __device__ __forceinline__ uint32_t sb() const { return h1 & 0xFFu; }
};
static_assert(sizeof(OpRec) == sizeof(DevOp), "OpRec mirrors DevOp");

// Payload element i of an operation, as T (i is a compile-time constant at
// every call site, so the record stays in scalar registers).
template <typename T>
__device__ __forceinline__ T pl(const OpRec &op, int i);
template <>
__device__ __forceinline__ double pl<double>(const OpRec &op, int i) {
    return __builtin_bit_cast(double, op.payload[i]);
}
template <>
__device__ __forceinline__ float pl<float>(const OpRec &op, int i) {
    return __builtin_bit_cast(float, (uint32_t)(op.payload[i >> 1] >> (32 * (i & 1))));
}
template <typename T>
__device__ __forceinline__ cpx<T> plc(const OpRec &op, int e) {
    return mk<T>(pl<T>(op, 2 * e), pl<T>(op, 2 * e + 1));
}

template <typename T>
struct PassTraits;
template <>
struct PassTraits<double> {
    static constexpr int R = kRegBitsC128;
    static constexpr int W = kThreadBitsC128;
};
template <>
struct PassTraits<float> {
    static constexpr int R = kRegBitsC64;
    static constexpr int W = kThreadBitsC64;
};

// Thread part of a layout: global-index bits and LDS slot index. Entries of
// thread bits at or above the workgroup's width are zero, so the loop runs
// over every possible bit without a data-dependent trip count.
template <int W>
__device__ __forceinline__ uint64_t thr_goff(const DevLayout &L, int tid) {
    uint64_t e[W];
#pragma unroll
    for (int b = 0; b < W; ++b) e[b] = L.thr_goff[b];
    // every entry in registers before the per-bit selects: the scalar loads
    // issue together instead of one after another inside per-bit branches
#pragma unroll
    for (int b = 0; b < W; ++b) asm volatile("" : : "s"(e[b]));
    uint64_t g = L.goff_xor;
#pragma unroll
    for (int b = 0; b < W; ++b) g ^= ((tid >> b) & 1) ? e[b] : 0ull;
    return g;
}
template <int W>
__device__ __forceinline__ uint32_t thr_slot(const DevLayout &L, int tid) {
    uint32_t e[W];
#pragma unroll
    for (int b = 0; b < W; ++b) e[b] = L.thr_slot[b];
#pragma unroll
    for (int b = 0; b < W; ++b) asm volatile("" : : "s"(e[b]));
    uint32_t sl = L.slot_xor;
#pragma unroll
    for (int b = 0; b < W; ++b) sl ^= ((tid >> b) & 1) ? e[b] : 0u;
    return sl;
}

// Slot index with bit `lo`-position removed (lo = 2^b - 1): the half-tile
// address of a slot whose bit b is fixed by the half being exchanged.
__device__ __forceinline__ uint32_t drop_bit(uint32_t x, uint32_t lo) {
    return (x & lo) | ((x >> 1) & ~lo);
}

// Register bit b of the i-th slot of a Gray-code walk over the register bits
// other than P (the walk flips one bit per step: bit ctz(i) of the reduced
// index).
template <int P>
__host__ __device__ constexpr int gray_bit(int i) {
    return __builtin_ctz(i) < P ? __builtin_ctz(i) : __builtin_ctz(i) + 1;
}
// Slot j visited at step i of that walk in half h.
template <int P>
__host__ __device__ constexpr int gray_slot(int i, int h) {
    const int g = i ^ (i >> 1);
    return ((g >> P) << (P + 1)) | (h << P) | (g & ((1 << P) - 1));
}

// Half-tile exchange, halves chosen by register bit P: every thread takes
// part in both halves with half of its registers. LDS byte addresses are the
// thread part XOR the per-register-bit generators (gw, gr), accumulated along
// a Gray-code walk, so only R generators stay live.
template <int P, typename T, int NR, int R>
__device__ __forceinline__ void exch_reg_halves(cpx<T> (&a)[NR], char *ldsb, uint32_t tw,
                                                const uint32_t (&gw)[R], uint32_t tr,
                                                const uint32_t (&gr)[R]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        __syncthreads();
        uint32_t aw = h ? tw ^ gw[P] : tw;
#pragma unroll
        for (int i = 0; i < NR / 2; ++i) {
            if (i) aw ^= gw[gray_bit<P>(i)];
            *reinterpret_cast<cpx<T> *>(ldsb + aw) = a[gray_slot<P>(i, h)];
        }
        __syncthreads();
        uint32_t ar = h ? tr ^ gr[P] : tr;
#pragma unroll
        for (int i = 0; i < NR / 2; ++i) {
            if (i) ar ^= gr[gray_bit<P>(i)];
            a[gray_slot<P>(i, h)] = *reinterpret_cast<const cpx<T> *>(ldsb + ar);
        }
    }
}

// Half-tile exchange, halves chosen by a thread bit: the threads whose bit is
// h move all of their registers in half h.
template <typename T, int NR, int R>
__device__ __forceinline__ void exch_thr_halves(cpx<T> (&a)[NR], char *ldsb, uint32_t tw,
                                                const uint32_t (&gw)[R], uint32_t tr,
                                                const uint32_t (&gr)[R], int mine) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        __syncthreads();
        if (mine == h) {
            uint32_t aw = tw;
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                if (i) aw ^= gw[__builtin_ctz(i)];
                *reinterpret_cast<cpx<T> *>(ldsb + aw) = a[i ^ (i >> 1)];
            }
        }
        __syncthreads();
        if (mine == h) {
            uint32_t ar = tr;
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                if (i) ar ^= gr[__builtin_ctz(i)];
                a[i ^ (i >> 1)] = *reinterpret_cast<const cpx<T> *>(ldsb + ar);
            }
        }
    }
}

__device__ __forceinline__ int src_bit(uint8_t src, int tid, uint64_t base) {
    const int pos = src & SRC_POS_MASK;
    return (src & ~SRC_POS_MASK) == SRC_THR ? (tid >> pos) & 1 : (int)((base >> pos) & 1);
}

// Global index of a tile's amplitude with all tile-local bits zero: the tile
// number with zeros inserted at the tile qubits (ascending). qv holds the
// pass's qubit list as aligned 32-bit words (scalar loads, not byte loads).
__device__ __forceinline__ uint64_t tile_base(const uint32_t (&qv)[7], int k, uint64_t tile) {
    uint64_t base = tile;
    // compile-time indices only: a run-time index into qv would put the
    // array in scratch memory
#pragma unroll
    for (int w = 0; w < 7; ++w) {
        const uint32_t word = qv[w];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (4 * w + j < k) {
                const int b = (word >> (8 * j)) & 0xFF;
                base = ((base >> b) << (b + 1)) | (base & ((1ull << b) - 1));
            }
        }
    }
    return base;
}

// Bring the pass's op records and layout tables into L2 with one vector load
// per 64-byte line: the interpreter then reads them one after another through
// the scalar cache without waiting on HBM. Returns a value for the caller to
// consume (after its tile loads are issued).
template <int W>
__device__ __forceinline__ uint32_t warm_records(const DevOp *opb, const DevPass &P, const DevLayout *LB,
                                                 int tid) {
    uint32_t warm = 0;
    const uint32_t *w = reinterpret_cast<const uint32_t *>(opb + P.op_begin);
    const uint32_t nw = (uint32_t)(P.op_end - P.op_begin) * (uint32_t)(sizeof(DevOp) / 4);
    for (uint32_t i = (uint32_t)tid * 16u; i < nw; i += (1u << W) * 16u) warm ^= w[i];
    const uint32_t *wl = reinterpret_cast<const uint32_t *>(LB);
    const uint32_t nl = (uint32_t)P.n_layouts * (uint32_t)(sizeof(DevLayout) / 4);
    for (uint32_t i = (uint32_t)tid * 16u; i < nl; i += (1u << W) * 16u) warm ^= wl[i];
    return warm;
}

// Load the thread's register slots of the tile at `base` in layout L. The
// global index of slot j is (base | thread part) XOR the register part,
// accumulated along a Gray-code walk over the register bits (the parts occupy
// disjoint bits), so only R per-bit offsets stay live.
template <typename T, int R, int W>
__device__ __forceinline__ void load_tile(cpx<T> (&a)[1 << R], const cpx<T> *st, const DevLayout &L,
                                          uint64_t base, int tid) {
    constexpr int NR = 1 << R;
    uint64_t idx = (base | thr_goff<W>(L, tid)) ^ L.reg_goff_xor;
    if (sizeof(T) == 4 && (L.flags & LAYOUT_PAIR_IO)) {
        // slots 2m and 2m + 1 are adjacent in memory (register bit 0 is
        // label 0): one 16-byte access; walk the other register bits.
        // Slots are written in the order of the single-slot walk below
        // (gray(2i) = 2 gray(i) + (i & 1)): stores in a different order
        // get merged across the two branches with a run-time slot address,
        // which puts the tile in scratch memory.
#pragma unroll
        for (int i = 0; i < NR / 2; ++i) {
            if (i) idx ^= L.reg_goff[__builtin_ctz(i) + 1];
            const int j = (i ^ (i >> 1)) << 1;
            cpx<float> a0, a1;
            ld_stream2(reinterpret_cast<const cpx<float> *>(st + idx), a0, a1);
            if (i & 1) {
                a[j + 1] = mk<T>((T)a1.x, (T)a1.y);
                a[j] = mk<T>((T)a0.x, (T)a0.y);
            } else {
                a[j] = mk<T>((T)a0.x, (T)a0.y);
                a[j + 1] = mk<T>((T)a1.x, (T)a1.y);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i) idx ^= L.reg_goff[__builtin_ctz(i)];
            a[i ^ (i >> 1)] = ld_stream(st + idx);
        }
    }
}

// On-demand Hadamard-layer amplitudes of H^M |j> in place of a load:
// 2^(-|M|/2) (-1)^popcount(i & j & M) where i agrees with j off M, else 0.
template <typename T, int R, int W>
__device__ __forceinline__ void generate_tile(cpx<T> (&a)[1 << R], const DevPass &P, const DevLayout &L,
                                              uint64_t base, int tid) {
    constexpr int NR = 1 << R;
    uint64_t idx = (base | thr_goff<W>(L, tid)) ^ L.reg_goff_xor;
    const uint64_t gm = P.gen_mask, gj = P.gen_j;
    const T mag = (T)P.gen_scale;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i) idx ^= L.reg_goff[__builtin_ctz(i)];
        const bool on = ((idx ^ gj) & ~gm) == 0;
        const T v = (__popcll(idx & gj & gm) & 1) ? -mag : mag;
        a[i ^ (i >> 1)] = mk<T>(on ? v : (T)0, (T)0);
    }
}

// On-demand product state in place of a load: amp[i] = prod_q u_q[bit q of i]
// with u_q = (u_q0, u_q1) read in FP64 from the pass's OP_GENP record and its
// continuation records (`gp` points at the OP_GENP record; n qubits, two per
// record). The factor of every qubit that no register bit holds is the same
// for all of the thread's slots: formed in FP64 and rounded once. The register
// bits' qubits then double a table over the slots.
template <typename T, int R, int W>
__device__ __forceinline__ void generate_product(cpx<T> (&a)[1 << R], const DevLayout &L, uint64_t base,
                                                 int tid, const OpRec *gp, int n) {
    const uint64_t idx0 = (base | thr_goff<W>(L, tid)) ^ L.reg_goff_xor;   // slot 0
    uint64_t regmask = 0;
#pragma unroll
    for (int p = 0; p < R; ++p) regmask |= L.reg_goff[p];
    cpx<double> c = mk<double>(1.0, 0.0);
    for (int q = 0; q < n; ++q) {
        if ((regmask >> q) & 1) continue;
        const OpRec &r = gp[q >> 1];
        const int e = (q & 1) * 4;
        const cpx<double> u0 = mk<double>(pl<double>(r, e), pl<double>(r, e + 1));
        const cpx<double> u1 = mk<double>(pl<double>(r, e + 2), pl<double>(r, e + 3));
        c = cmul(c, ((idx0 >> q) & 1) ? u1 : u0);
    }
    a[0] = mk<T>((T)c.x, (T)c.y);
#pragma unroll
    for (int p = 0; p < R; ++p) {
        const int q = __builtin_ctzll(L.reg_goff[p]);
        const OpRec &r = gp[q >> 1];
        const int e = (q & 1) * 4;
        const cpx<T> u0 = mk<T>((T)pl<double>(r, e), (T)pl<double>(r, e + 1));
        const cpx<T> u1 = mk<T>((T)pl<double>(r, e + 2), (T)pl<double>(r, e + 3));
        // slot 0 has bit q of idx0; a slot with register bit p set has the other
        const bool b0 = (idx0 >> q) & 1;
        const cpx<T> lo = b0 ? u1 : u0, hi = b0 ? u0 : u1;
#pragma unroll
        for (int j = 0; j < (1 << p); ++j) {
            a[j | (1 << p)] = cmul(a[j], hi);
            a[j] = cmul(a[j], lo);
        }
    }
}

template <typename T, int R, int W>
__device__ __forceinline__ void store_tile(const cpx<T> (&a)[1 << R], cpx<T> *st, const DevLayout &L,
                                           uint64_t base, int tid) {
    constexpr int NR = 1 << R;
    uint64_t idx = (base | thr_goff<W>(L, tid)) ^ L.reg_goff_xor;
    if (sizeof(T) == 4 && (L.flags & LAYOUT_PAIR_IO)) {
#pragma unroll
        for (int i = 0; i < NR / 2; ++i) {
            if (i) idx ^= L.reg_goff[__builtin_ctz(i) + 1];
            const int j = (i ^ (i >> 1)) << 1;
            st_stream2(reinterpret_cast<cpx<float> *>(st + idx), mk<float>((float)a[j].x, (float)a[j].y),
                       mk<float>((float)a[j + 1].x, (float)a[j + 1].y));
        }
    } else {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i) idx ^= L.reg_goff[__builtin_ctz(i)];
            st_stream(st + idx, a[i ^ (i >> 1)]);
        }
    }
}

// The pass's operation list on one register tile: a host-built program read
// record by record (the next one prefetched) through the scalar cache.
// D2: the variant that also executes OP_DENSE2 (its 4x4 needs many more
// registers; passes without it run the lean variant). FX: exchanges move the
// whole tile through a full-tile LDS buffer (2 barriers each instead of 4).
template <typename T, bool D2, bool FX>
__device__ __forceinline__ void run_ops(cpx<T> (&a)[1 << PassTraits<T>::R], const DevOp *opb, int oi,
                                        const int oe, const DevLayout *LB, const uint64_t base,
                                        const int tid, char *const ldsb) {
    constexpr int R = PassTraits<T>::R;
    constexpr int W = PassTraits<T>::W;
    constexpr int NR = 1 << R;
    constexpr int SH = sizeof(T) == 8 ? 4 : 3;   // log2 of the slot size in bytes
    cpx<T> f = mk<T>((T)1, (T)0);   // per-thread diagonal factor (OP_UDN)
    if (oi < oe) {
        const OpRec *recs = reinterpret_cast<const OpRec *>(opb);
        OpRec op = recs[oi];
        for (;;) {
            OpRec nxt = recs[oi + 1 < oe ? oi + 1 : oi];   // prefetch the next record
            switch (op.code()) {
            case OP_EXCH: {
                const DevLayout &Lw = LB[op.a()], &Lr = LB[op.b()];
                if constexpr (FX) {
                    // every register at once: slot addresses without a half bit
                    uint32_t aw = thr_slot<W>(Lw, tid) << SH, ar = thr_slot<W>(Lr, tid) << SH;
                    uint32_t gw[R], gr[R];
#pragma unroll
                    for (int b = 0; b < R; ++b) {
                        gw[b] = Lw.reg_slot[b] << SH;
                        gr[b] = Lr.reg_slot[b] << SH;
                    }
                    __syncthreads();   // the previous exchange's reads are done
#pragma unroll
                    for (int i = 0; i < NR; ++i) {
                        if (i) aw ^= gw[__builtin_ctz(i)];
                        *reinterpret_cast<cpx<T> *>(ldsb + aw) = a[i ^ (i >> 1)];
                    }
                    __syncthreads();
#pragma unroll
                    for (int i = 0; i < NR; ++i) {
                        if (i) ar ^= gr[__builtin_ctz(i)];
                        a[i ^ (i >> 1)] = *reinterpret_cast<const cpx<T> *>(ldsb + ar);
                    }
                    break;
                }
                const uint32_t lo = (1u << op.sb()) - 1u;
                uint32_t tw = thr_slot<W>(Lw, tid), tr = thr_slot<W>(Lr, tid), gw[R], gr[R];
                tw = drop_bit(tw, lo) << SH;
                tr = drop_bit(tr, lo) << SH;
#pragma unroll
                for (int b = 0; b < R; ++b) {
                    gw[b] = drop_bit(Lw.reg_slot[b], lo) << SH;
                    gr[b] = drop_bit(Lr.reg_slot[b], lo) << SH;
                }
                if ((op.sa() & ~SRC_POS_MASK) == SRC_REG) {
                    SV_SWITCH_A(op.sa() & SRC_POS_MASK, exch_reg_halves<PA>(a, ldsb, tw, gw, tr, gr))
                } else {
                    exch_thr_halves(a, ldsb, tw, gw, tr, gr, (tid >> (op.sa() & SRC_POS_MASK)) & 1);
                }
                break;
            }
            case OP_D1H: {
                const cpx<T> d = plc<T>(op, 0);
                if (op.b()) {
                    SV_SWITCH_A(op.a(), r_d1_half<PA, 1>(a, d))
                } else {
                    SV_SWITCH_A(op.a(), r_d1_half<PA, 0>(a, d))
                }
                break;
            }
            case OP_D2Q: {
                // the quarter of the slots with bit a == xa and bit b == xb,
                // both bits and both values at compile time (with bit b at
                // run time the multiply covers the half and selects)
                const cpx<T> d = plc<T>(op, 0);
#define SV_D2Q(XA, XB) \
    SV_SWITCH_A(op.a(), SV_SWITCH_B(op.b(), if constexpr (PA != PB) r_d1_quarter<PA, XA, PB, XB>(a, d)))
                switch (op.sa() & 3u) {
                case 0: SV_D2Q(0, 0) break;
                case 1: SV_D2Q(1, 0) break;
                case 2: SV_D2Q(0, 1) break;
                default: SV_D2Q(1, 1) break;
                }
#undef SV_D2Q
                break;
            }
            case OP_D1HU: {
                // under an execution mask: threads (and, for tile-base or
                // upper thread bits, whole waves) whose bit does not match skip
                const cpx<T> d = plc<T>(op, 0);
                const bool on = src_bit(op.sa(), tid, base) == ((op.b() >> 1) & 1);
                if (on) {
                    if (op.b() & 1) {
                        SV_SWITCH_A(op.a(), r_d1_half<PA, 1>(a, d))
                    } else {
                        SV_SWITCH_A(op.a(), r_d1_half<PA, 0>(a, d))
                    }
                }
                break;
            }
            case OP_RPERM: {   // emitted only in passes with OP_DENSE2
                if constexpr (D2) {
                    SV_SWITCH_A(op.a(), SV_SWITCH_B(op.b(), if constexpr (PA != PB) r_rperm<PA, PB>(a)))
                }
                break;
            }
            case OP_DENSE2: {
                if constexpr (!D2) break;
                // 4x4 on register bits 1 and 0; its 16 entries continue in the
                // payloads of the OP_CONT records that follow
                constexpr int PER = sizeof(T) == 8 ? 4 : 8;
                constexpr int NC = 16 / PER - 1;
                cpx<T> m[16];
#pragma unroll
                for (int e = 0; e < PER; ++e) m[e] = plc<T>(op, e);
#pragma unroll
                for (int t = 0; t < NC; ++t) {
                    const OpRec &c = recs[oi + 1 + t];
#pragma unroll
                    for (int e = 0; e < PER; ++e) m[PER * (t + 1) + e] = plc<T>(c, e);
                }
#pragma unroll
                for (int j0 = 0; j0 < NR; j0 += 4) {
                    const cpx<T> x0 = a[j0], x1 = a[j0 + 1], x2 = a[j0 + 2], x3 = a[j0 + 3];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        a[j0 + r] = cadd(cmul2(m[4 * r], x0, m[4 * r + 1], x1),
                                         cmul2(m[4 * r + 2], x2, m[4 * r + 3], x3));
                }
                oi += NC;   // skip the continuation records
                nxt = recs[oi + 1 < oe ? oi + 1 : oi];
                break;
            }
            case OP_D1R: {
                const cpx<T> d0 = cmul(f, plc<T>(op, 0)), d1 = cmul(f, plc<T>(op, 1));
                f = mk<T>((T)1, (T)0);
                SV_SWITCH_A(op.a(), r_d1_reg<PA>(a, d0, d1))
                break;
            }
            case OP_UDN: {
                // merged diagonals on thread / tile-base bits: C times the
                // ratio of every term whose bit (or bit pair) is set
                cpx<T> g = plc<T>(op, 0);
                constexpr int UDT = sizeof(T) == 8 ? kMaxUdTermsC128 : kMaxUdTerms;
#pragma unroll
                for (int i = 0; i < UDT; ++i) {
                    if (i >= (int)op.a()) break;
                    const uint8_t s1 = i < 4 ? (uint8_t)(op.data >> (16 * i)) : op.sa();
                    const uint8_t s2 = i < 4 ? (uint8_t)(op.data >> (16 * i + 8)) : op.sb();
                    const int on = src_bit(s1, tid, base) & (s2 == kNoSource ? 1 : src_bit(s2, tid, base));
                    const cpx<T> r = plc<T>(op, i + 1);
                    g = on ? cmul(g, r) : g;
                }
                f = cmul(f, g);
                break;
            }
            case OP_APPLYF: {
                r_mul_all(a, f);
                f = mk<T>((T)1, (T)0);
                break;
            }
            case OP_DENSE1: {
                cpx<T> g00 = plc<T>(op, 0), g01 = plc<T>(op, 1);
                cpx<T> g10 = plc<T>(op, 2), g11 = plc<T>(op, 3);
                if (op.b()) {
                    g00 = cmul(f, g00);
                    g01 = cmul(f, g01);
                    g10 = cmul(f, g10);
                    g11 = cmul(f, g11);
                    f = mk<T>((T)1, (T)0);
                }
                SV_SWITCH_A(op.a(), r_dense1<PA>(a, g00, g01, g10, g11))
                break;
            }
            case OP_DENSE1RI: {
                const T r00 = pl<T>(op, 0), r01 = pl<T>(op, 1), r10 = pl<T>(op, 2), r11 = pl<T>(op, 3);
#define SV_RI(F) \
    case F: SV_SWITCH_A(op.a(), (r_dense1_ri<PA, ((F) & 1), (((F) >> 1) & 1), ((F) >> 2)>(a, r00, r01, r10, r11))) break;
                switch (op.b()) {
                    SV_RI(0) SV_RI(1) SV_RI(2) SV_RI(3) SV_RI(4) SV_RI(5) SV_RI(6) SV_RI(7)
                    default: break;
                }
#undef SV_RI
                break;
            }
            case OP_H: {
                // consecutive Hadamards on different register bits share one
                // record: one dispatch for the whole run
#pragma unroll
                for (int bb = 0; bb < R; ++bb)
                    if ((op.a() >> bb) & 1u) {
                        SV_SWITCH_A(bb, r_h<PA>(a))
                    }
                break;
            }
            case OP_X: {
                SV_SWITCH_A(op.a(), r_x<PA>(a))
                break;
            }
            case OP_CXR: {
                SV_SWITCH_A(op.a(), SV_SWITCH_B(op.b(), if constexpr (PA != PB) r_cx_reg<PA, PB>(a)))
                break;
            }
            case OP_CXU: {
                const bool c = src_bit(op.sa(), tid, base) != 0;
                SV_SWITCH_A(op.a(), r_cx_uni<PA>(a, c))
                break;
            }
            case OP_CXT: {
                if ((base >> (op.sa() & SRC_POS_MASK)) & 1) {
                    SV_SWITCH_A(op.a(), r_x<PA>(a))
                }
                break;
            }
            case OP_CCX: {
                // thread / tile-base controls: the threads whose bits do not
                // match skip (execution mask); register controls pick slots
                const uint32_t uv = (uint32_t)(op.data >> 8) & 3u;
                bool on = true;
                if (op.sa() != kNoSource) on = on && src_bit(op.sa(), tid, base) == (int)(uv & 1u);
                if (op.sb() != kNoSource) on = on && src_bit(op.sb(), tid, base) == (int)(uv >> 1);
                if (on) {
                    const uint32_t cm = op.b(), cv = (uint32_t)op.data & 0xFFu;
                    SV_SWITCH_A(op.a(), r_ccx<PA>(a, cm, cv))
                }
                break;
            }
            case OP_MARK: {
                if (base == op.data && tid == (int)(op.sa() | (op.sb() << 8))) {
#pragma unroll
                    for (int j = 0; j < NR; ++j)
                        if (j == (int)op.a()) a[j] = mk<T>(-a[j].x, -a[j].y);
                }
                break;
            }
            case OP_SCALE: {
                r_scale(a, pl<T>(op, 0));
                break;
            }
            default:
                break;
            }
            if (++oi >= oe) break;
            op = nxt;
        }
    }
}

// One workgroup per tile (grid: tiles x batch). FX: full-tile exchanges, for
// launches too small to fill the chip, where the pass is latency-bound and LDS
// does not limit occupancy. GEN: the pass generates its input (a Hadamard
// layer or basis state, or a product state) instead of loading it; only a
// circuit's first pass does, and the generating code lives in its own variant
// so that it does not weigh on the register allocation of the others.
// One tile of a pass: load it (or generate it), run the pass's operations,
// store it. `st` is the state, `opb` its op records, `tile` the tile number.
// The plan records never alias the state (restrict): the compiler may then
// read them with scalar loads even when their addresses come from memory.
template <typename T, bool D2, bool FX, bool GEN>
__device__ __forceinline__ void pass_tile(cpx<T> *__restrict__ st, const DevPass *__restrict__ Pp,
                                          const DevLayout *__restrict__ LB, const DevOp *__restrict__ opb,
                                          uint64_t tile, int tid, char *const ldsb) {
    const DevPass &P = *Pp;
    constexpr int R = PassTraits<T>::R;
    constexpr int W = PassTraits<T>::W;
    constexpr int NR = 1 << R;
    const uint32_t *qw = reinterpret_cast<const uint32_t *>(P.q);
    uint32_t qv[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) qv[i] = qw[i];
#pragma unroll
    for (int i = 0; i < 7; ++i) asm volatile("" : : "s"(qv[i]));   // one batch of scalar loads
    const uint64_t base = tile_base(qv, P.k, tile);

    const uint32_t warm = warm_records<W>(opb, P, LB, tid);
    cpx<T> a[NR];
    int op_first = P.op_begin;
    if constexpr (GEN) {
        if (P.flags & PASS_GEN_PRODUCT) {
            // the OP_GENP record and its continuations hold the product data
            const OpRec *gp = reinterpret_cast<const OpRec *>(opb) + P.op_begin;
            generate_product<T, R, W>(a, LB[0], base, tid, gp, gp->a());
            op_first += 1 + (int)gp->b();
        } else {
            generate_tile<T, R, W>(a, P, LB[0], base, tid);
        }
    } else {
        load_tile<T, R, W>(a, st, LB[0], base, tid);
    }
    asm volatile("" : : "v"(warm));   // the warming loads complete before the ops

    run_ops<T, D2, FX>(a, opb, op_first, P.op_end, LB, base, tid, ldsb);

    if (P.flags & PASS_SYNC_STORE) __syncthreads();
    store_tile<T, R, W>(a, st, LB[P.store_layout], base, tid);
}

template <typename T, bool D2, bool FX, bool GEN>
__global__ __launch_bounds__(1 << PassTraits<T>::W) void k_pass(cpx<T> *__restrict__ state, uint64_t n_amps,
                                              const DevPass *__restrict__ passes, int pass_idx,
                                              const DevLayout *__restrict__ layouts,
                                              const DevOp *__restrict__ ops, uint64_t ops_stride) {
    constexpr int R = PassTraits<T>::R;
    constexpr int W = PassTraits<T>::W;
    constexpr int NR = 1 << R;
    __shared__ cpx<T> lds[FX ? (NR << W) : (NR << W) / 2];   // a tile, or half a tile
    const DevPass &P = passes[pass_idx];
    pass_tile<T, D2, FX, GEN>(state + (uint64_t)blockIdx.y * n_amps, &P, layouts + P.layout_begin,
                              ops + (uint64_t)blockIdx.y * ops_stride, xcd_tile(blockIdx.x, gridDim.x),
                              threadIdx.x, reinterpret_cast<char *>(lds));
}

// One pass of several independent states with their own plans (continuous
// batching): workgroup b runs tile items[b].tile of the pass reqs[items[b].req]
// names on that request's state. Each tile's arithmetic is the same as in
// k_pass, so a state's result does not depend on what else shares a launch.
// The plan records are addressed inside `arena` (a restrict argument, never
// written by the kernel), which lets them be read through the scalar cache.
template <typename T, bool D2, bool FX, bool GEN>
__global__ __launch_bounds__(1 << PassTraits<T>::W) void k_pass_multi(const char *__restrict__ arena,
                                                                      const StepReq *__restrict__ reqs,
                                                                      const StepItem *__restrict__ items) {
    constexpr int R = PassTraits<T>::R;
    constexpr int W = PassTraits<T>::W;
    constexpr int NR = 1 << R;
    __shared__ cpx<T> lds[FX ? (NR << W) : (NR << W) / 2];
    const StepItem it = items[blockIdx.x];
    const StepReq &rq = reqs[it.req];
    const DevPass *P = reinterpret_cast<const DevPass *>(arena + rq.passes_off) + rq.pass;
    const DevLayout *LB = reinterpret_cast<const DevLayout *>(arena + rq.layouts_off) + P->layout_begin;
    const DevOp *ops = reinterpret_cast<const DevOp *>(arena + rq.ops_off);
    pass_tile<T, D2, FX, GEN>(reinterpret_cast<cpx<T> *>(rq.state), P, LB, ops, it.tile, threadIdx.x,
                              reinterpret_cast<char *>(lds));
}

// Persistent variant for launches larger than the chip holds at once. Each
// workgroup walks a sequence of (batch entry, tile) items and issues the loads
// of its next tile before it runs the current tile's operations, so that its
// own HBM traffic overlaps its arithmetic (one workgroup per tile runs its
// load, ops and store one after another, and the workgroups sharing a CU
// drift into the same phase: all loading, then all computing). Two tiles sit
// in registers (about 170 VGPRs: three waves per SIMD). FX: exchanges through
// a full-tile LDS buffer (2 barriers each, two workgroups per CU by LDS) or a
// half-tile one (4 barriers each, three workgroups per CU). Items are split into 8 contiguous eighths, one
// per XCD (workgroup g runs on XCD g mod 8), when grid and item count allow.
// Every workgroup leaves its loop after a bounded number of items. Passes that
// generate their input do not run here.
template <typename T, bool FX>
__global__ __launch_bounds__(1 << PassTraits<T>::W) __attribute__((amdgpu_waves_per_eu(2)))
void k_pass_pipe(cpx<T> *__restrict__ state, uint64_t n_amps, const DevPass *__restrict__ passes,
                 int pass_idx, const DevLayout *__restrict__ layouts, const DevOp *__restrict__ ops,
                 uint64_t ops_stride, uint64_t n_items) {
    constexpr int R = PassTraits<T>::R;
    constexpr int W = PassTraits<T>::W;
    constexpr int NR = 1 << R;
    __shared__ cpx<T> lds[FX ? (NR << W) : (NR << W) / 2];
    char *const ldsb = reinterpret_cast<char *>(lds);

    const DevPass &P = passes[pass_idx];
    const int tid = threadIdx.x;
    const DevLayout *LB = layouts + P.layout_begin;
    const uint32_t *qw = reinterpret_cast<const uint32_t *>(P.q);
    uint32_t qv[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) qv[i] = qw[i];
#pragma unroll
    for (int i = 0; i < 7; ++i) asm volatile("" : : "s"(qv[i]));
    const int tshift = __builtin_ctzll(P.tiles);   // tiles is a power of two
    const uint64_t tmask = P.tiles - 1;

    const uint32_t G = gridDim.x, g = blockIdx.x;
    uint64_t it, step, limit;
    if ((G & 7u) == 0 && (n_items & 7u) == 0) {
        const uint64_t eighth = n_items >> 3;
        it = (uint64_t)(g & 7u) * eighth + (g >> 3);
        step = G >> 3;
        limit = (uint64_t)(g & 7u) * eighth + eighth;
    } else {
        it = g;
        step = G;
        limit = n_items;
    }
    if (it >= limit) return;

    cpx<T> *st = state + (it >> tshift) * n_amps;
    const DevOp *opb = ops + (it >> tshift) * ops_stride;
    uint64_t base = tile_base(qv, P.k, it & tmask);
    const uint32_t warm = warm_records<W>(opb, P, LB, tid);
    // The register tile `a` is only ever written by register moves and
    // arithmetic, never directly by loads (the first tile goes through `b`
    // too): with loads in flight into `a` at the op loop's entry, the
    // compiler's wait counting would put full waits inside the op handlers,
    // and in later iterations those would also wait for the prefetch and the
    // previous tile's stores.
    cpx<T> a[NR], b[NR];
    load_tile<T, R, W>(b, st, LB[0], base, tid);
#pragma unroll
    for (int j = 0; j < NR; ++j) a[j] = b[j];
    asm volatile("" : : "v"(warm));

    for (;;) {
        const uint64_t nit = it + step;
        const bool more = nit < limit;
        cpx<T> *nst = st;
        const DevOp *nopb = opb;
        uint64_t nbase = base;
        if (more) {
            nst = state + (nit >> tshift) * n_amps;
            nopb = ops + (nit >> tshift) * ops_stride;
            nbase = tile_base(qv, P.k, nit & tmask);
            load_tile<T, R, W>(b, nst, LB[0], nbase, tid);   // in flight during the ops
        }
        run_ops<T, false, FX>(a, opb, P.op_begin, P.op_end, LB, base, tid, ldsb);
        if (P.flags & PASS_SYNC_STORE) __syncthreads();
        store_tile<T, R, W>(a, st, LB[P.store_layout], base, tid);
        if (!more) break;
#pragma unroll
        for (int j = 0; j < NR; ++j) a[j] = b[j];
        it = nit;
        st = nst;
        opb = nopb;
        base = nbase;
    }
}

// ---------------------------------------------------------------------------
// Whole state in one workgroup's LDS; one operation at a time.

__device__ __forceinline__ uint32_t ins0(uint32_t x, int q) {
    return ((x >> q) << (q + 1)) | (x & ((1u << q) - 1));
}

// Bring a small plan's op records and the first constant of every op that has
// constants into L2, all threads at once: the op loop then reads them one op
// at a time without waiting on HBM. Returns a value to be consumed.
template <typename T>
__device__ __forceinline__ T small_warm(const SmallOp *ops, int n_ops, const T *cst, int tid, int nt) {
    T w = (T)0;
    for (int oi = tid; oi < n_ops; oi += nt) {
        const SmallOp o = ops[oi];
        const bool has_consts = o.code == SOP_D1 || o.code == SOP_D2 || o.code == SOP_DENSE1 ||
                                o.code == SOP_DENSE2 || o.code == SOP_SCALE;
        if (has_consts) w += cst[o.data];
    }
    return w;
}

template <typename T>
__global__ __launch_bounds__(256) void k_small(cpx<T> *__restrict__ state, int n,
                                               const SmallOp *__restrict__ ops, int n_ops,
                                               const T *__restrict__ consts,
                                               uint64_t const_stride) {
    constexpr int kCap = sizeof(T) == 8 ? (1 << kSmallMaxQubitsC128) : (1 << kSmallMaxQubitsC64);
    __shared__ cpx<T> s[kCap];
    const uint32_t N = 1u << n;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    cpx<T> *st = state + (uint64_t)blockIdx.x * N;
    const T *cst = consts + (uint64_t)blockIdx.x * const_stride;
    const T warm = small_warm(ops, n_ops, cst, tid, nt);
    for (uint32_t i = tid; i < N; i += nt) s[i] = st[i];
    asm volatile("" : : "v"(warm));   // the warming loads complete before the ops
    __syncthreads();
    for (int oi = 0; oi < n_ops; ++oi) {
        const SmallOp op = ops[oi];
        const int q0 = op.q0, q1 = op.q1;
        const T *c = cst + op.data;
        switch (op.code) {
        case SOP_D1:
            for (uint32_t i = tid; i < N; i += nt) s[i] = cmul(s[i], ldc(c + 2 * ((i >> q0) & 1)));
            break;
        case SOP_D2:
            for (uint32_t i = tid; i < N; i += nt)
                s[i] = cmul(s[i], ldc(c + 2 * ((((i >> q0) & 1) << 1) | ((i >> q1) & 1))));
            break;
        case SOP_MARK:
            if (tid == 0) {
                const uint32_t m = (uint32_t)op.data;
                s[m] = mk<T>(-s[m].x, -s[m].y);
            }
            break;
        case SOP_DENSE1: {
            const cpx<T> g00 = ldc(c), g01 = ldc(c + 2), g10 = ldc(c + 4), g11 = ldc(c + 6);
            for (uint32_t p = tid; p < N / 2; p += nt) {
                const uint32_t i0 = ins0(p, q0), i1 = i0 | (1u << q0);
                const cpx<T> x0 = s[i0], x1 = s[i1];
                s[i0] = cmul2(g00, x0, g01, x1);
                s[i1] = cmul2(g10, x0, g11, x1);
            }
            break;
        }
        case SOP_DENSE2: {
            const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
            for (uint32_t p = tid; p < N / 4; p += nt) {
                const uint32_t b = ins0(ins0(p, lo), hi);
                const uint32_t ii[4] = {b, b | (1u << q1), b | (1u << q0), b | (1u << q0) | (1u << q1)};
                cpx<T> x[4];
#pragma unroll
                for (int l = 0; l < 4; ++l) x[l] = s[ii[l]];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const T *row = c + 8 * r;
                    s[ii[r]] = cadd(cmul2(ldc(row), x[0], ldc(row + 2), x[1]),
                                    cmul2(ldc(row + 4), x[2], ldc(row + 6), x[3]));
                }
            }
            break;
        }
        case SOP_X:
            for (uint32_t p = tid; p < N / 2; p += nt) {
                const uint32_t i0 = ins0(p, q0), i1 = i0 | (1u << q0);
                const cpx<T> t = s[i0];
                s[i0] = s[i1];
                s[i1] = t;
            }
            break;
        case SOP_Y:
            for (uint32_t p = tid; p < N / 2; p += nt) {
                const uint32_t i0 = ins0(p, q0), i1 = i0 | (1u << q0);
                const cpx<T> x0 = s[i0], x1 = s[i1];
                s[i0] = mk<T>(x1.y, -x1.x);
                s[i1] = mk<T>(-x0.y, x0.x);
            }
            break;
        case SOP_CX: {  // q0 = control, q1 = target
            const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
            for (uint32_t p = tid; p < N / 4; p += nt) {
                const uint32_t b = ins0(ins0(p, lo), hi) | (1u << q0);
                const uint32_t i1 = b | (1u << q1);
                const cpx<T> t = s[b];
                s[b] = s[i1];
                s[i1] = t;
            }
            break;
        }
        case SOP_CCX: {  // q0, q1 = controls, q2 = target
            const int q2 = op.q2;
            int lo = q0 < q1 ? q0 : q1, mid = q0 < q1 ? q1 : q0, hi = q2;
            if (hi < mid) { const int t = hi; hi = mid; mid = t; }
            if (mid < lo) { const int t = mid; mid = lo; lo = t; }
            for (uint32_t p = tid; p < N / 8; p += nt) {
                const uint32_t b = ins0(ins0(ins0(p, lo), mid), hi) | (1u << q0) | (1u << q1);
                const uint32_t i1 = b | (1u << q2);
                const cpx<T> t = s[b];
                s[b] = s[i1];
                s[i1] = t;
            }
            break;
        }
        case SOP_SWAP: {
            const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
            for (uint32_t p = tid; p < N / 4; p += nt) {
                const uint32_t b = ins0(ins0(p, lo), hi);
                const uint32_t i01 = b | (1u << q1), i10 = b | (1u << q0);
                const cpx<T> t = s[i01];
                s[i01] = s[i10];
                s[i10] = t;
            }
            break;
        }
        case SOP_SCALE: {
            const T f = c[0];
            for (uint32_t i = tid; i < N; i += nt) s[i] = mk<T>(s[i].x * f, s[i].y * f);
            break;
        }
        default:
            break;
        }
        __syncthreads();
    }
    for (uint32_t i = tid; i < N; i += nt) st[i] = s[i];
}

// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_fill_basis(cpx<T> *__restrict__ state, uint64_t n_amps,
                                                    uint64_t total, uint64_t j) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const uint64_t r = i & (n_amps - 1);   // n_amps is a power of two
        state[i] = mk<T>(r == j ? (T)1 : (T)0, (T)0);
    }
}

// Fixed-shape FP64 reduction. Stage 1: block `blk` of state `b` sums the
// contiguous chunk [blk * chunk, (blk + 1) * chunk): each thread strides
// through it in order, then a fixed tree over the 256 threads. Stage 2: one
// block per state sums the partials with the same fixed pattern.
constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_tree_sum(double v, double *sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    return sh[0];
}

// One block's share of a readout: sum of |a_i|^2 (1 - 2 bit q of i, or 1 for
// q < 0) over [lo, lo + chunk), each thread striding in a fixed order, then
// the fixed tree. Every load is 16 bytes: one complex128 amplitude, or two
// adjacent complex64 ones (chunks are even; the state is 16-byte aligned).
template <typename T>
__device__ __forceinline__ double block_readout(const cpx<T> *__restrict__ st, uint64_t lo, uint64_t chunk,
                                                int qubit, double *sh) {
    double acc = 0.0;
    if constexpr (sizeof(T) == 8) {
#pragma unroll 4
        for (uint64_t i = lo + threadIdx.x; i < lo + chunk; i += kRedThreads) {
            const cpx<T> v = ld_stream(st + i);
            const double p = v.x * v.x + v.y * v.y;
            acc += (qubit >= 0 && ((i >> qubit) & 1)) ? -p : p;
        }
    } else {
        const uint64_t hi = lo + chunk;
#pragma unroll 4
        for (uint64_t i = lo + 2 * threadIdx.x; i < hi; i += 2 * kRedThreads) {
            cpx<float> v0, v1;
            if (i + 1 < hi) {
                ld_stream2(st + i, v0, v1);
            } else {   // a one-amplitude chunk (n = 0 is not a state; kept for safety)
                v0 = st[i];
                v1 = mk<float>(0.f, 0.f);
            }
            const double p0 = (double)v0.x * (double)v0.x + (double)v0.y * (double)v0.y;
            const double p1 = (double)v1.x * (double)v1.x + (double)v1.y * (double)v1.y;
            acc += (qubit >= 0 && ((i >> qubit) & 1)) ? -p0 : p0;
            acc += (qubit >= 0 && (((i + 1) >> qubit) & 1)) ? -p1 : p1;
        }
    }
    return block_tree_sum(acc, sh);
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_reduce_partial(const cpx<T> *__restrict__ state,
                                                                uint64_t n_amps, uint64_t chunk,
                                                                int qubit, double *__restrict__ part,
                                                                int nblk) {
    __shared__ double sh[kRedThreads];
    const cpx<T> *st = state + (uint64_t)blockIdx.y * n_amps;
    const double s = block_readout<T>(st, (uint64_t)blockIdx.x * chunk, chunk, qubit, sh);
    if (threadIdx.x == 0) part[(uint64_t)blockIdx.y * nblk + blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double *__restrict__ part,
                                                              int nblk, double *__restrict__ out) {
    __shared__ double sh[kRedThreads];
    const double *p = part + (uint64_t)blockIdx.x * nblk;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kRedThreads) acc += p[i];
    const double s = block_tree_sum(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Several states' readouts in one launch (continuous batching): each work
// item is one block of k_reduce_partial's decomposition of its state, summed
// in the same order, so a request's result equals its single-state readout.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_reduce_multi(const RedItem *__restrict__ items,
                                                              double *__restrict__ part) {
    __shared__ double sh[kRedThreads];
    const RedItem it = items[blockIdx.x];
    const double s = block_readout<T>(static_cast<const cpx<T> *>(it.state), (uint64_t)it.blk * it.chunk, it.chunk,
                                      it.qubit, sh);
    if (threadIdx.x == 0) part[it.part] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_final_multi(const FinItem *__restrict__ items,
                                                             const double *__restrict__ part,
                                                             double *__restrict__ out) {
    __shared__ double sh[kRedThreads];
    const FinItem it = items[blockIdx.x];
    const double *p = part + it.first;
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < it.count; i += kRedThreads) acc += p[i];
    const double s = block_tree_sum(acc, sh);
    if (threadIdx.x == 0) out[it.slot] = s;
}

template <typename T>
__global__ void k_gather(const cpx<T> *__restrict__ state, const uint64_t *__restrict__ idx,
                         uint64_t k, double *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) {
        const cpx<T> v = state[idx[i]];
        out[2 * i] = (double)v.x;
        out[2 * i + 1] = (double)v.y;
    }
}

// ---------------------------------------------------------------------------
// Serving: many independent small circuits in one launch, one workgroup per
// request; the state never leaves LDS and the result is <Z_qubit> in FP64.

template <typename T>
__device__ __forceinline__ void small_apply(cpx<T> *s, uint32_t N, const SmallOp &op, const T *c,
                                            int tid, int nt) {
    const int q0 = op.q0, q1 = op.q1;
    switch (op.code) {
    case SOP_D1:
        for (uint32_t i = tid; i < N; i += nt) s[i] = cmul(s[i], ldc(c + 2 * ((i >> q0) & 1)));
        break;
    case SOP_D2:
        for (uint32_t i = tid; i < N; i += nt)
            s[i] = cmul(s[i], ldc(c + 2 * ((((i >> q0) & 1) << 1) | ((i >> q1) & 1))));
        break;
    case SOP_MARK:
        if (tid == 0) {
            const uint32_t m = (uint32_t)op.data;
            s[m] = mk<T>(-s[m].x, -s[m].y);
        }
        break;
    case SOP_DENSE1: {
        const cpx<T> g00 = ldc(c), g01 = ldc(c + 2), g10 = ldc(c + 4), g11 = ldc(c + 6);
        for (uint32_t p = tid; p < N / 2; p += nt) {
            const uint32_t i0 = ins0(p, q0), i1 = i0 | (1u << q0);
            const cpx<T> x0 = s[i0], x1 = s[i1];
            s[i0] = cmul2(g00, x0, g01, x1);
            s[i1] = cmul2(g10, x0, g11, x1);
        }
        break;
    }
    case SOP_DENSE2: {
        const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
        for (uint32_t p = tid; p < N / 4; p += nt) {
            const uint32_t b = ins0(ins0(p, lo), hi);
            const uint32_t ii[4] = {b, b | (1u << q1), b | (1u << q0), b | (1u << q0) | (1u << q1)};
            cpx<T> x[4];
#pragma unroll
            for (int l = 0; l < 4; ++l) x[l] = s[ii[l]];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const T *row = c + 8 * r;
                s[ii[r]] = cadd(cmul2(ldc(row), x[0], ldc(row + 2), x[1]),
                                cmul2(ldc(row + 4), x[2], ldc(row + 6), x[3]));
            }
        }
        break;
    }
    case SOP_X:
        for (uint32_t p = tid; p < N / 2; p += nt) {
            const uint32_t i0 = ins0(p, q0), i1 = i0 | (1u << q0);
            const cpx<T> t = s[i0];
            s[i0] = s[i1];
            s[i1] = t;
        }
        break;
    case SOP_Y:
        for (uint32_t p = tid; p < N / 2; p += nt) {
            const uint32_t i0 = ins0(p, q0), i1 = i0 | (1u << q0);
            const cpx<T> x0 = s[i0], x1 = s[i1];
            s[i0] = mk<T>(x1.y, -x1.x);
            s[i1] = mk<T>(-x0.y, x0.x);
        }
        break;
    case SOP_CX: {
        const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
        for (uint32_t p = tid; p < N / 4; p += nt) {
            const uint32_t b = ins0(ins0(p, lo), hi) | (1u << q0);
            const uint32_t i1 = b | (1u << q1);
            const cpx<T> t = s[b];
            s[b] = s[i1];
            s[i1] = t;
        }
        break;
    }
    case SOP_CCX: {  // q0, q1 = controls, q2 = target
        const int q2 = op.q2;
        int lo = q0 < q1 ? q0 : q1, mid = q0 < q1 ? q1 : q0, hi = q2;
        if (hi < mid) { const int t = hi; hi = mid; mid = t; }
        if (mid < lo) { const int t = mid; mid = lo; lo = t; }
        for (uint32_t p = tid; p < N / 8; p += nt) {
            const uint32_t b = ins0(ins0(ins0(p, lo), mid), hi) | (1u << q0) | (1u << q1);
            const uint32_t i1 = b | (1u << q2);
            const cpx<T> t = s[b];
            s[b] = s[i1];
            s[i1] = t;
        }
        break;
    }
    case SOP_SWAP: {
        const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
        for (uint32_t p = tid; p < N / 4; p += nt) {
            const uint32_t b = ins0(ins0(p, lo), hi);
            const uint32_t i01 = b | (1u << q1), i10 = b | (1u << q0);
            const cpx<T> t = s[i01];
            s[i01] = s[i10];
            s[i10] = t;
        }
        break;
    }
    default:
        break;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_small_jobs(const SmallJob *__restrict__ jobs,
                                                    const SmallOp *__restrict__ ops,
                                                    const T *__restrict__ consts,
                                                    double *__restrict__ out) {
    constexpr int kCap = sizeof(T) == 8 ? (1 << kSmallMaxQubitsC128) : (1 << kSmallMaxQubitsC64);
    __shared__ cpx<T> s[kCap];
    __shared__ double red[kRedThreads];
    const SmallJob J = jobs[blockIdx.x];
    const uint32_t N = 1u << J.n;
    const int tid = threadIdx.x, nt = blockDim.x;
    const T *cst = consts + J.const_begin;
    const T warm = small_warm(ops + J.op_begin, J.n_ops, cst, tid, nt);
    for (uint32_t i = tid; i < N; i += nt) s[i] = mk<T>(i == 0 ? (T)1 : (T)0, (T)0);
    asm volatile("" : : "v"(warm));   // the warming loads complete before the ops
    __syncthreads();
    for (int oi = 0; oi < J.n_ops; ++oi) {
        const SmallOp op = ops[J.op_begin + oi];
        small_apply<T>(s, N, op, cst + op.data, tid, nt);
        __syncthreads();
    }
    // <Z_qubit> in FP64: each thread in index order, then a fixed tree
    double acc = 0.0;
    for (uint32_t i = tid; i < N; i += nt) {
        const double re = (double)s[i].x, im = (double)s[i].y;
        const double p = re * re + im * im;
        acc += ((i >> J.qubit) & 1) ? -p : p;
    }
    const double z = block_tree_sum(acc, red);
    if (tid == 0) out[blockIdx.x] = z;
}

// ---------------------------------------------------------------------------
// Adjoint differentiation helpers.

// lambda_b = Z_q psi_b for every batch entry (psi at state, lambda at out).
template <typename T>
__global__ __launch_bounds__(256) void k_copy_z(const cpx<T> *__restrict__ psi, cpx<T> *__restrict__ lam,
                                                uint64_t total, uint64_t n_amps, int q) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        // bit q of the index within its state (states are 2^n apart, q < n)
        const cpx<T> v = psi[i];
        lam[i] = ((i >> q) & 1) ? mk<T>(-v.x, -v.y) : v;
    }
}

// Block sum with a fixed order (wave butterflies, then the waves in order);
// the result is valid in thread 0 only, and the scratch is free on return.
template <int NTH = kRedThreads>
__device__ __forceinline__ double block_sum_t0(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NTH / 64; ++w) s += sh[w];
    __syncthreads();
    return s;
}

constexpr int kIpSub = 4096;   // amplitudes staged per sub-chunk (2^12)

// The terms' contributions at global index i, staged slot j (psi_i = buf[j]):
// Z terms use bit q of i; X and Y terms take their partner from slot j ^ 2^q,
// where q is then the qubit's bit position inside the staged sub-chunk.
// ZT = false: Z terms are left to the caller (summed per thread, see
// k_pauli_ip_sub).
template <int MT, typename T, bool ZT = true>
__device__ __forceinline__ void ip_terms_at(double (&acc)[MT], uint64_t i, uint32_t j, cpx<T> l,
                                            const cpx<T> *buf, const IpTerms &terms, int nt) {
    const cpx<T> v = buf[j];
    const double lx = (double)l.x, ly = (double)l.y;
    const double base = lx * (double)v.y - ly * (double)v.x;   // Im(conj(l) v)
#pragma clang loop unroll(full)
    for (int t = 0; t < MT; ++t) {
        if (t >= nt) continue;   // predicated: acc stays in registers
        const uint32_t m = 1u << terms.q[t];
        if (terms.pauli[t] == 3) {
            if constexpr (ZT) acc[t] += ((i >> terms.q[t]) & 1) ? -base : base;
        } else {
            const cpx<T> w = buf[j ^ m];
            double px = (double)w.x, py = (double)w.y;
            if (terms.pauli[t] == 2) {   // Y: (-i, +i) psi_{i ^ m} for bit 0, 1
                const double sgn = (j & m) ? 1.0 : -1.0;
                px = -sgn * (double)w.y;
                py = sgn * (double)w.x;
            }
            acc[t] += lx * py - ly * px;
        }
    }
}

// Several Im <lambda_b | P_t | psi_b> in one read of psi and lambda. The
// chunk is walked in sub-chunks of kIpSub amplitudes staged in LDS: Z terms
// take any qubit; X and Y terms take qubits whose partner i ^ 2^q lies in the
// same sub-chunk. It serves complex64 and states below 2^12 amplitudes;
// k_pauli_ip_sub serves the rest and X and Y terms on higher qubits. Stage 1
// per (chunk, batch entry); part[(b * nt + t) * nblk + chunk].
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_pauli_ip_multi(const cpx<T> *__restrict__ psi,
                                                                const cpx<T> *__restrict__ lam,
                                                                uint64_t n_amps, uint64_t chunk,
                                                                IpTerms terms, int nt,
                                                                double *__restrict__ part, int nblk) {
    __shared__ cpx<T> buf[kIpSub];
    __shared__ double sh[kRedThreads / 64];
    const cpx<T> *ps = psi + (uint64_t)blockIdx.y * n_amps;
    const cpx<T> *lm = lam + (uint64_t)blockIdx.y * n_amps;
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    const uint32_t sub = chunk < (uint64_t)kIpSub ? (uint32_t)chunk : (uint32_t)kIpSub;
    double acc[kMaxIpTerms];
#pragma clang loop unroll(full)
    for (int t = 0; t < kMaxIpTerms; ++t) acc[t] = 0.0;
    for (uint64_t s0 = lo; s0 < lo + chunk; s0 += sub) {
        __syncthreads();   // the previous sub-chunk's reads are done
        for (uint32_t j = threadIdx.x; j < sub; j += kRedThreads) buf[j] = ps[s0 + j];
        __syncthreads();
        // lambda one step ahead: the next load is in flight during the terms
        uint32_t j = threadIdx.x;
        cpx<T> l = j < sub ? lm[s0 + j] : mk<T>((T)0, (T)0);
        for (; j < sub; j += kRedThreads) {
            const uint32_t jn = j + kRedThreads;
            const cpx<T> ln = jn < sub ? lm[s0 + jn] : l;
            ip_terms_at<kMaxIpTerms>(acc, s0 + j, j, l, buf, terms, nt);
            l = ln;
        }
    }
#pragma clang loop unroll(full)
    for (int t = 0; t < kMaxIpTerms; ++t) {
        if (t >= nt) continue;
        const double sum = block_sum_t0(acc[t], sh);
        if (threadIdx.x == 0) part[((uint64_t)blockIdx.y * nt + t) * nblk + blockIdx.x] = sum;
    }
}

// The same sums over sub-chunks that need not be contiguous: a sub-chunk is
// the 2^12 amplitudes whose bits outside
// B = {0, .., lb - 1} u {hq[0], .., hq[h - 1]} (lb = 12 - h, 0 <= h <= 8) are
// fixed. Its slot j holds bit k < lb of j at qubit k and bit lb + k at qubit
// hq[k], so an X or Y term on a qubit of B finds its partner inside the staged
// sub-chunk (terms.q of an X or Y term is the qubit's bit position in B; of a
// Z term, the qubit; Z terms only with h = 0). The nxy <= MXY X and Y terms
// come first in `terms`, the Z terms after them. psi and lambda are both
// staged in LDS by TH threads, and the next sub-chunk's loads are in flight
// while the current one is summed. Block blockIdx.x walks sub-chunks
// [x * per, (x + 1) * per) of the 2^(n - 12), per <= 2^kIpZw; the partial
// layout matches k_pauli_ip_multi's.
//
// With j = r * TH + tid, the sign of a Z term (its bit of i) is a thread bit,
// a bit of r, or a bit of the sub-chunk's base, and in the last case a bit of
// the block's local sub-chunk number or the same for the whole block. So the
// Z terms need no accumulators of their own: the thread keeps the total of
// Im(conj(l) v), its signed sums over each bit of r and over each bit of the
// local sub-chunk number, and each Z term takes the matching one.
// (complex128 with more than 8 X / Y terms: 512, for the registers; LDS
// holds one complex128 block per CU either way)
constexpr int kIpSubThreadsC128 = 1024;
constexpr int kIpSubThreadsC64 = 1024;
constexpr int kIpZw = 4;            // bits of the local sub-chunk number
template <typename T, int MXY, int TH>
__global__ __launch_bounds__(TH) void k_pauli_ip_sub(const cpx<T> *__restrict__ psi,
                                                    const cpx<T> *__restrict__ lam, uint64_t n_amps,
                                                    uint64_t per, IpTerms terms, int nt, int nxy, IpHiMap map,
                                                    double *__restrict__ part, int nblk) {
    constexpr int NRS = kIpSub / TH;              // slots per thread: j = r * TH + tid
    constexpr int RB = __builtin_ctz(NRS);        // bits of r: bits log2(TH) .. 11 of j
    constexpr int TB = __builtin_ctz(TH);         // thread bits of j
    static_assert((TH & (TH - 1)) == 0 && TH >= 256 && TH <= 1024, "thread count");
    __shared__ cpx<T> buf[kIpSub], lbuf[kIpSub];
    __shared__ double sh[kMaxIpTerms * (TH / 64)];
    const cpx<T> *ps = psi + (uint64_t)blockIdx.y * n_amps;
    const cpx<T> *lm = lam + (uint64_t)blockIdx.y * n_amps;
    const int h = map.h, lb = 12 - h;
    // global offset of slot j: the bits of j deposited on B (OR-linear in j)
    auto dep = [&](uint32_t j) {
        uint64_t o = j & ((1u << lb) - 1u);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < h) o |= (uint64_t)((j >> (lb + k)) & 1u) << map.hq[k];
        return o;
    };
    const uint64_t toff = dep(threadIdx.x);
    uint64_t gr[RB];   // offsets of the register-slot bits of j
#pragma unroll
    for (int b = 0; b < RB; ++b) gr[b] = dep((uint32_t)TH << b);
    double acc[MXY];
#pragma unroll
    for (int t = 0; t < MXY; ++t) acc[t] = 0.0;
    double ztot = 0.0, zr[RB], zw[kIpZw];
#pragma unroll
    for (int k = 0; k < RB; ++k) zr[k] = 0.0;
#pragma unroll
    for (int k = 0; k < kIpZw; ++k) zw[k] = 0.0;
    // the sub-chunk's base index: its number with zeros inserted at B
    auto base_of = [&](uint64_t sc) {
        uint64_t b = sc << lb;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < h) {
                const int q = map.hq[k];
                b = ((b >> q) << (q + 1)) | (b & ((1ull << q) - 1));
            }
        return b;
    };
    auto slot_off = [&](int r) {
        uint64_t o = toff;
#pragma unroll
        for (int b = 0; b < RB; ++b) o |= ((r >> b) & 1) ? gr[b] : 0ull;
        return o;
    };
    // software pipeline: the next sub-chunk's loads are in flight while the
    // current one is summed from LDS
    const uint64_t s_beg = (uint64_t)blockIdx.x * per, s_end = s_beg + per;
    // amplitudes in flight as 2-vectors (register arrays of plain vectors)
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 *psv = reinterpret_cast<const v2 *>(ps), *lmv = reinterpret_cast<const v2 *>(lm);
    v2 *bufv = reinterpret_cast<v2 *>(buf), *lbufv = reinterpret_cast<v2 *>(lbuf);
    v2 pv[NRS], lv[NRS];
    {
        const uint64_t b0 = base_of(s_beg);
#pragma clang loop unroll(full)
        for (int r = 0; r < NRS; ++r) {
            pv[r] = psv[b0 | slot_off(r)];
            lv[r] = lmv[b0 | slot_off(r)];
        }
    }
    for (uint64_t sc = s_beg; sc < s_end; ++sc) {
#pragma clang loop unroll(full)
        for (int r = 0; r < NRS; ++r) {
            bufv[r * TH + threadIdx.x] = pv[r];
            lbufv[r * TH + threadIdx.x] = lv[r];
        }
        // the thread's own slots, from the registers before the prefetch
        // reuses them: lambda in FP64 for the X and Y terms, and the Z sums
        double lx[NRS], ly[NRS];
        double z0 = 0.0;
#pragma unroll
        for (int r = 0; r < NRS; ++r) {
            lx[r] = (double)lv[r].x;
            ly[r] = (double)lv[r].y;
            const double b = lx[r] * (double)pv[r].y - ly[r] * (double)pv[r].x;   // Im(conj(l) v)
            z0 += b;
#pragma unroll
            for (int k = 0; k < RB; ++k) zr[k] += ((r >> k) & 1) ? -b : b;
        }
        ztot += z0;
        const uint32_t u = (uint32_t)(sc - s_beg);   // the local sub-chunk number
#pragma unroll
        for (int k = 0; k < kIpZw; ++k) zw[k] += ((u >> k) & 1u) ? -z0 : z0;
        __syncthreads();
        {   // the last sub-chunk reloads itself (cache hits) instead of a branch
            const uint64_t b1 = base_of(sc + 1 < s_end ? sc + 1 : sc);
#pragma clang loop unroll(full)
            for (int r = 0; r < NRS; ++r) {
                pv[r] = psv[b1 | slot_off(r)];
                lv[r] = lmv[b1 | slot_off(r)];
            }
        }
        // X and Y terms: Im(conj(l_j) (P psi)_j) with the partner slot
        // j ^ m, m = 2^q. X gives lx wy - ly wx; Y gives s (lx wx + ly wy)
        // with s = +1 where bit q of j is set, else -1. A bit q below TB is
        // a thread bit: the partner is slot r of thread tid ^ m and s is the
        // same for all of the thread's slots (applied once per sub-chunk);
        // otherwise q is a bit of r: the partner is slot r ^ (m / TH) of this
        // thread and s is uniform over the block.
#pragma clang loop unroll(full)
        for (int t = 0; t < MXY; ++t) {
            if (t >= nxy) continue;   // a uniform branch: acc stays in registers
            const int pa = terms.pauli[t];
            const uint32_t m = 1u << terms.q[t];
            double s = 0.0;
            if (m < (uint32_t)TH) {
                const cpx<T> *pb = buf + (threadIdx.x ^ m);
                if (pa == 1) {
#pragma unroll
                    for (int r = 0; r < NRS; ++r) {
                        const cpx<T> w = pb[r * TH];
                        s += lx[r] * (double)w.y - ly[r] * (double)w.x;
                    }
                    acc[t] += s;
                } else {
#pragma unroll
                    for (int r = 0; r < NRS; ++r) {
                        const cpx<T> w = pb[r * TH];
                        s += lx[r] * (double)w.x + ly[r] * (double)w.y;
                    }
                    acc[t] += (threadIdx.x & m) ? s : -s;
                }
            } else {
                const uint32_t rm = m / (uint32_t)TH;
                const cpx<T> *pb = buf + threadIdx.x;
                if (pa == 1) {
#pragma unroll
                    for (int r = 0; r < NRS; ++r) {
                        const cpx<T> w = pb[(r ^ rm) * TH];
                        s += lx[r] * (double)w.y - ly[r] * (double)w.x;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < NRS; ++r) {
                        const cpx<T> w = pb[(r ^ rm) * TH];
                        const double p = lx[r] * (double)w.x + ly[r] * (double)w.y;
                        s += ((uint32_t)r & rm) ? p : -p;
                    }
                }
                acc[t] += s;
            }
            // one term at a time: reads of later terms hoisted above this
            // point would hold registers the accumulators need
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();   // every read of this sub-chunk is done before the next is staged
    }
    // Z term on qubit q (h = 0, so bit q of i is bit q of j for q < 12 and
    // bit q - 12 of the sub-chunk number above): the matching sum. Every
    // term's block sum at once: a butterfly per wave, one barrier, then
    // thread t adds term t's wave sums in order (the arithmetic of
    // block_sum_t0, term by term).
    const uint64_t sb = s_beg;
#pragma clang loop unroll(full)
    for (int t = 0; t < kMaxIpTerms; ++t) {
        if (t >= nt) continue;
        double v;
        if (t < MXY && t < nxy) {
            v = acc[t < MXY ? t : 0];
        } else {
            const int q = terms.q[t];
            if (q < TB) {
                v = ((threadIdx.x >> q) & 1u) ? -ztot : ztot;
            } else if (q < 12) {
                v = 0.0;
#pragma unroll
                for (int k = 0; k < RB; ++k)
                    if (q - TB == k) v = zr[k];
            } else if (q - 12 < kIpZw && (1ull << (q - 12)) < per) {
                v = 0.0;
#pragma unroll
                for (int k = 0; k < kIpZw; ++k)
                    if (q - 12 == k) v = zw[k];
            } else {
                v = ((sb >> (q - 12)) & 1u) ? -ztot : ztot;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & 63) == 0) sh[t * (TH / 64) + (threadIdx.x >> 6)] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nt) {
        double s = 0.0;
        for (int w = 0; w < TH / 64; ++w) s += sh[threadIdx.x * (TH / 64) + w];
        part[((uint64_t)blockIdx.y * nt + threadIdx.x) * nblk + blockIdx.x] = s;
    }
}

// Stage 2: one block per batch entry adds each term's chunk sums, in order,
// to out[b * out_stride + off[t]] (terms sharing a parameter add in turn).
__global__ __launch_bounds__(kRedThreads) void k_accumulate_multi(const double *__restrict__ part, int nblk,
                                                                  int nt, double *__restrict__ out,
                                                                  uint64_t out_stride, IpOffsets offs) {
    __shared__ double sh[kRedThreads / 64];
    const uint64_t b = blockIdx.x;
    for (int t = 0; t < nt; ++t) {
        const double *p = part + (b * nt + t) * nblk;
        double acc = 0.0;
        for (int i = threadIdx.x; i < nblk; i += kRedThreads) acc += p[i];
        const double s = block_sum_t0(acc, sh);
        if (threadIdx.x == 0) out[b * out_stride + offs.off[t]] += s;
    }
}

// ---------------------------------------------------------------------------
// Launchers

hipError_t launch_fill_basis(int dt, void *state, uint64_t n_amps, int batch, uint64_t j,
                             hipStream_t st) {
    const uint64_t total = n_amps * (uint64_t)batch;
    uint64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (dt == 2)
        hipLaunchKernelGGL(k_fill_basis<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (cpx<double> *)state, n_amps, total, j);
    else
        hipLaunchKernelGGL(k_fill_basis<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (cpx<float> *)state, n_amps, total, j);
    return hipGetLastError();
}

// Launches of at most this many workgroups (two per CU) use full-tile exchanges.
constexpr uint64_t kFullExchangeMaxBlocks = 512;

// Workgroups of the persistent pass kernel that fit on the device at once
// (occupancy x compute units), per precision; looked up once.
template <typename T, bool FX>
static hipError_t pipe_grid(uint64_t *out) {
    static std::mutex mu;
    static uint64_t cached = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (!cached) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void *>(&k_pass_pipe<T, FX>), 1 << PassTraits<T>::W, 0);
        if (e != hipSuccess) return e;
        if (per_cu < 1 || cus < 1) return hipErrorInvalidConfiguration;
        cached = (uint64_t)per_cu * (uint64_t)cus;
    }
    *out = cached;
    return hipSuccess;
}

hipError_t launch_pass(int dt, void *state, uint64_t n_amps, int batch, const DevPass *d_passes,
                       int pass_idx, const DevPass &h_pass, const DevLayout *d_layouts,
                       const DevOp *d_ops, uint64_t ops_stride, int pipeline, hipStream_t st) {
    // The kernel is compiled for one tile geometry per precision; a pass that
    // does not match it is refused before launch.
    const int R = dt == 2 ? kRegBitsC128 : kRegBitsC64;
    const int W = dt == 2 ? kThreadBitsC128 : kThreadBitsC64;
    if (h_pass.w < kMinThreadBits || h_pass.w > W || h_pass.k != h_pass.w + R ||
        h_pass.tiles != (n_amps >> h_pass.k) || (h_pass.tiles << h_pass.k) != n_amps ||
        (h_pass.tiles & (h_pass.tiles - 1)) != 0)
        return hipErrorInvalidValue;
    const dim3 block(1u << h_pass.w);
    const bool d2 = (h_pass.flags & PASS_DENSE2) != 0;
    const uint64_t items = h_pass.tiles * (uint64_t)batch;
    const bool fx = items <= kFullExchangeMaxBlocks;
    const bool gen = (h_pass.flags & PASS_GENERATES) != 0;
    if (pipeline && !d2 && !fx && !gen && h_pass.w == W) {
        // persistent: as many workgroups as fit at once (a multiple of 8,
        // so that each XCD walks its own eighth of the items)
        const bool full = pipeline == 2;
        uint64_t grid = 0;
        hipError_t e = dt == 2 ? (full ? pipe_grid<double, true>(&grid) : pipe_grid<double, false>(&grid))
                               : (full ? pipe_grid<float, true>(&grid) : pipe_grid<float, false>(&grid));
        if (e != hipSuccess) return e;
        if (grid >= 8) grid &= ~(uint64_t)7;
        if (grid > items) grid = items;
#define SV_PIPE(TT, FXV)                                                                                  \
    hipLaunchKernelGGL((k_pass_pipe<TT, FXV>), dim3((unsigned)grid), block, 0, st, (cpx<TT> *)state, n_amps, \
                       d_passes, pass_idx, d_layouts, d_ops, ops_stride, items)
        if (dt == 2) {
            if (full) SV_PIPE(double, true);
            else SV_PIPE(double, false);
        } else {
            if (full) SV_PIPE(float, true);
            else SV_PIPE(float, false);
        }
#undef SV_PIPE
        return hipGetLastError();
    }
    const dim3 grid((unsigned)h_pass.tiles, (unsigned)batch);
#define SV_PASS(TT, D2V, FXV)                                                                              \
    do {                                                                                                   \
        if (gen)                                                                                           \
            hipLaunchKernelGGL((k_pass<TT, D2V, FXV, true>), grid, block, 0, st, (cpx<TT> *)state, n_amps,  \
                               d_passes, pass_idx, d_layouts, d_ops, ops_stride);                          \
        else                                                                                               \
            hipLaunchKernelGGL((k_pass<TT, D2V, FXV, false>), grid, block, 0, st, (cpx<TT> *)state, n_amps, \
                               d_passes, pass_idx, d_layouts, d_ops, ops_stride);                          \
    } while (0)
    if (dt == 2) {
        if (d2) {
            if (fx) SV_PASS(double, true, true);
            else SV_PASS(double, true, false);
        } else {
            if (fx) SV_PASS(double, false, true);
            else SV_PASS(double, false, false);
        }
    } else {
        if (d2) {
            if (fx) SV_PASS(float, true, true);
            else SV_PASS(float, true, false);
        } else {
            if (fx) SV_PASS(float, false, true);
            else SV_PASS(float, false, false);
        }
    }
#undef SV_PASS
    return hipGetLastError();
}

hipError_t launch_pass_multi(int dt, const void *d_arena, const StepReq *d_reqs, const StepItem *d_items,
                             uint32_t n_items, bool gen, bool d2, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    // always the half-tile exchange variant: a request runs the same code
    // whatever the size of the launch it shares
    const dim3 grid(n_items), block(1u << (dt == 2 ? kThreadBitsC128 : kThreadBitsC64));
#define SV_MULTI(TT, D2V, GV) \
    hipLaunchKernelGGL((k_pass_multi<TT, D2V, false, GV>), grid, block, 0, st, (const char *)d_arena, d_reqs, d_items)
    if (dt == 2) {
        if (d2) {
            if (gen) SV_MULTI(double, true, true);
            else SV_MULTI(double, true, false);
        } else {
            if (gen) SV_MULTI(double, false, true);
            else SV_MULTI(double, false, false);
        }
    } else {
        if (d2) {
            if (gen) SV_MULTI(float, true, true);
            else SV_MULTI(float, true, false);
        } else {
            if (gen) SV_MULTI(float, false, true);
            else SV_MULTI(float, false, false);
        }
    }
#undef SV_MULTI
    return hipGetLastError();
}

hipError_t launch_reduce_multi(int dt, const RedItem *d_items, uint32_t n_items, double *d_part,
                               const FinItem *d_fin, uint32_t n_fin, double *d_out, hipStream_t st) {
    if (n_items == 0 || n_fin == 0) return hipSuccess;
    if (dt == 2)
        hipLaunchKernelGGL(k_reduce_multi<double>, dim3(n_items), dim3(kRedThreads), 0, st, d_items, d_part);
    else
        hipLaunchKernelGGL(k_reduce_multi<float>, dim3(n_items), dim3(kRedThreads), 0, st, d_items, d_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_final_multi, dim3(n_fin), dim3(kRedThreads), 0, st, d_fin, (const double *)d_part, d_out);
    return hipGetLastError();
}

size_t reduce_chunk(int n) { return (size_t)((1ull << n) / (uint64_t)reduce_blocks(n)); }

hipError_t launch_small(int dt, void *state, int n, int batch, const SmallOp *d_ops, int n_ops,
                        const void *d_consts, uint64_t const_stride, hipStream_t st) {
    const uint32_t N = 1u << n;
    const unsigned threads = N >= 512 ? 256u : (N / 2 >= 64 ? N / 2 : 64u);
    if (dt == 2)
        hipLaunchKernelGGL(k_small<double>, dim3(batch), dim3(threads), 0, st,
                           (cpx<double> *)state, n, d_ops, n_ops, (const double *)d_consts,
                           const_stride);
    else
        hipLaunchKernelGGL(k_small<float>, dim3(batch), dim3(threads), 0, st,
                           (cpx<float> *)state, n, d_ops, n_ops, (const float *)d_consts,
                           const_stride);
    return hipGetLastError();
}

// Number of stage-1 blocks per state: a function of n only (determinism).
int reduce_blocks(int n) {
    if (n <= 12) return 1;
    const int b = n - 12;               // chunks of 4096 amplitudes ...
    return 1 << (b < 10 ? b : 10);      // ... at most 1024 blocks
}

size_t reduce_partials_size(int n) { return (size_t)reduce_blocks(n); }

// blocks of the sub-chunk inner products: 16 sub-chunks of 2^12 each
size_t pauli_ip_partials_size(int n) {
    const size_t sub = n >= 16 ? (size_t)1 << (n - 16) : 1;
    const size_t red = reduce_partials_size(n);
    return sub > red ? sub : red;
}

hipError_t launch_reduce(int dt, const void *state, int n, int batch, int qubit,
                         double *d_partials, double *d_out, hipStream_t st) {
    const uint64_t N = 1ull << n;
    const int nblk = reduce_blocks(n);
    const uint64_t chunk = N / (uint64_t)nblk;
    if (dt == 2)
        hipLaunchKernelGGL(k_reduce_partial<double>, dim3(nblk, batch), dim3(kRedThreads), 0, st,
                           (const cpx<double> *)state, N, chunk, qubit, d_partials, nblk);
    else
        hipLaunchKernelGGL(k_reduce_partial<float>, dim3(nblk, batch), dim3(kRedThreads), 0, st,
                           (const cpx<float> *)state, N, chunk, qubit, d_partials, nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(batch), dim3(kRedThreads), 0, st,
                       (const double *)d_partials, nblk, d_out);
    return hipGetLastError();
}

// Partial sums of the allocation-free readout: a file-scope device array, so
// that the entry point using it never allocates. Each GPU holds its own copy
// until the process ends, and every such call on a GPU shares it.
static __device__ __align__(256) double scratch[kStaticPartials];

hipError_t static_partials(double **out) {
    // Host code must not pass the array's name to a kernel (it names a
    // host-side stand-in): take the device address once per device, with that
    // device current, and use that address from then on.
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        double *p = nullptr;
        e = hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

hipError_t launch_gather(int dt, const void *state, const uint64_t *d_idx, size_t k,
                         double *d_out, hipStream_t st) {
    if (k == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((k + 255) / 256);
    if (dt == 2)
        hipLaunchKernelGGL(k_gather<double>, dim3(blocks), dim3(256), 0, st,
                           (const cpx<double> *)state, d_idx, (uint64_t)k, d_out);
    else
        hipLaunchKernelGGL(k_gather<float>, dim3(blocks), dim3(256), 0, st,
                           (const cpx<float> *)state, d_idx, (uint64_t)k, d_out);
    return hipGetLastError();
}

hipError_t launch_copy_z(int dt, const void *psi, void *lam, uint64_t n_amps, int batch, int q,
                         hipStream_t st) {
    const uint64_t total = n_amps * (uint64_t)batch;
    uint64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (dt == 2)
        hipLaunchKernelGGL(k_copy_z<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (const cpx<double> *)psi, (cpx<double> *)lam, total, n_amps, q);
    else
        hipLaunchKernelGGL(k_copy_z<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (const cpx<float> *)psi, (cpx<float> *)lam, total, n_amps, q);
    return hipGetLastError();
}

static hipError_t launch_pauli_ip_sub(int dt, const void *psi, const void *lam, int n, int batch,
                                      const IpTerms &terms, const IpOffsets &offs, int nt, const IpHiMap &map,
                                      double *d_partials, double *d_grad, uint64_t grad_stride, hipStream_t st);

hipError_t launch_pauli_ip_multi(int dt, const void *psi, const void *lam, int n, int batch,
                                 const IpTerms &terms, const IpOffsets &offs, int nt, double *d_partials,
                                 double *d_grad, uint64_t grad_stride, hipStream_t st) {
    if (nt <= 0) return hipSuccess;
    if (nt > kMaxIpTerms) return hipErrorInvalidValue;
    if (n >= 12) {
        // contiguous 2^12-amplitude sub-chunks (h = 0) of the pipelined kernel
        IpHiMap map{};
        return launch_pauli_ip_sub(dt, psi, lam, n, batch, terms, offs, nt, map, d_partials, d_grad, grad_stride,
                                   st);
    }
    const uint64_t N = 1ull << n;
    const int nblk = reduce_blocks(n);
    const uint64_t chunk = N / (uint64_t)nblk;
    const uint64_t sub = chunk < (uint64_t)kIpSub ? chunk : (uint64_t)kIpSub;
    for (int t = 0; t < nt; ++t)   // partners must stay inside the staged sub-chunk
        if (terms.q[t] >= n || (terms.pauli[t] != 3 && (1ull << terms.q[t]) >= sub)) return hipErrorInvalidValue;
    if (dt == 2)
        hipLaunchKernelGGL(k_pauli_ip_multi<double>, dim3(nblk, batch), dim3(kRedThreads), 0, st,
                           (const cpx<double> *)psi, (const cpx<double> *)lam, N, chunk, terms, nt, d_partials,
                           nblk);
    else
        hipLaunchKernelGGL(k_pauli_ip_multi<float>, dim3(nblk, batch), dim3(kRedThreads), 0, st,
                           (const cpx<float> *)psi, (const cpx<float> *)lam, N, chunk, terms, nt, d_partials,
                           nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_accumulate_multi, dim3(batch), dim3(kRedThreads), 0, st, (const double *)d_partials,
                       nblk, nt, d_grad, grad_stride, offs);
    return hipGetLastError();
}

// Sub-chunk sums (k_pauli_ip_sub) for n >= 12 and 0 <= h <= 8.
static hipError_t launch_pauli_ip_sub(int dt, const void *psi, const void *lam, int n, int batch,
                                      const IpTerms &terms, const IpOffsets &offs, int nt, const IpHiMap &map,
                                      double *d_partials, double *d_grad, uint64_t grad_stride, hipStream_t st) {
    if (nt <= 0) return hipSuccess;
    if (nt > kMaxIpTerms || n < 12 || n > 62 || map.h < 0 || map.h > 8) return hipErrorInvalidValue;
    const int lb = 12 - map.h;
    for (int k = 0; k < map.h; ++k)   // ascending, above the low bits, inside the state
        if (map.hq[k] < lb || map.hq[k] >= n || (k && map.hq[k] <= map.hq[k - 1])) return hipErrorInvalidValue;
    // the X and Y terms first (their accumulators), then the Z terms (only
    // with contiguous sub-chunks); the order of the terms changes no sum
    int nxy = 0;
    for (int t = 0; t < nt; ++t) {
        const int pa = terms.pauli[t];
        if (pa < 1 || pa > 3 || terms.q[t] >= (pa == 3 ? n : 12) || (pa == 3 && map.h != 0))
            return hipErrorInvalidValue;
        nxy += pa != 3;
    }
    if (nxy > kIpMaxXYTerms) return hipErrorInvalidValue;
    IpTerms tt{};
    IpOffsets oo{};
    int w = 0;
    for (int z = 0; z < 2; ++z)
        for (int t = 0; t < nt; ++t)
            if ((terms.pauli[t] == 3) == (z == 1)) {
                tt.q[w] = terms.q[t];
                tt.pauli[w] = terms.pauli[t];
                oo.off[w] = offs.off[t];
                ++w;
            }
    const uint64_t N = 1ull << n;
    // up to 2^kIpZw sub-chunks per block, but at least 32 blocks per state
    // where it has that many sub-chunks (a function of n alone, so that a
    // term's summation order does not depend on the batch)
    const uint64_t nsc = N >> 12;
    const uint64_t nblk64 = std::max(nsc >> kIpZw, std::min<uint64_t>(nsc, 32));
    const uint64_t per = nsc / nblk64;
    if (nblk64 > (uint64_t)pauli_ip_partials_size(n)) return hipErrorInvalidValue;
    const int nblk = (int)nblk64;
    const dim3 grid(nblk, batch);
    const bool few = nxy <= kMaxIpHiTerms;   // fewer accumulators, fewer registers
#define SV_IP_SUB(TT, MTT, THH)                                                                   \
    hipLaunchKernelGGL((k_pauli_ip_sub<TT, MTT, THH>), grid, dim3(THH), 0, st, (const cpx<TT> *)psi, \
                       (const cpx<TT> *)lam, N, per, tt, nt, nxy, map, d_partials, nblk)
    if (dt == 2) {
        if (few) SV_IP_SUB(double, kMaxIpHiTerms, kIpSubThreadsC128);
        else SV_IP_SUB(double, kIpMaxXYTerms, kIpSubThreadsC128 / 2);   // 12 FP64 accumulators: 512 threads
    } else {
        if (few) SV_IP_SUB(float, kMaxIpHiTerms, kIpSubThreadsC64);
        else SV_IP_SUB(float, kIpMaxXYTerms, kIpSubThreadsC64);
    }
#undef SV_IP_SUB
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_accumulate_multi, dim3(batch), dim3(kRedThreads), 0, st, (const double *)d_partials,
                       nblk, nt, d_grad, grad_stride, oo);
    return hipGetLastError();
}

hipError_t launch_pauli_ip_hi(int dt, const void *psi, const void *lam, int n, int batch,
                              const IpTerms &terms, const IpOffsets &offs, int nt, const IpHiMap &map,
                              double *d_partials, double *d_grad, uint64_t grad_stride, hipStream_t st) {
    if (nt > kMaxIpHiTerms || n < 13 || map.h < 1) return hipErrorInvalidValue;
    for (int t = 0; t < nt; ++t)
        if (terms.pauli[t] == 3) return hipErrorInvalidValue;
    return launch_pauli_ip_sub(dt, psi, lam, n, batch, terms, offs, nt, map, d_partials, d_grad, grad_stride, st);
}

int pauli_ip_multi_chunk_bits(int n) {
    const uint64_t chunk = (1ull << n) / (uint64_t)reduce_blocks(n);
    const uint64_t sub = chunk < (uint64_t)kIpSub ? chunk : (uint64_t)kIpSub;
    return 63 - __builtin_clzll(sub);
}

hipError_t launch_small_jobs(int dt, const SmallJob *d_jobs, int n_jobs, const SmallOp *d_ops,
                             const void *d_consts, double *d_out, hipStream_t st) {
    if (n_jobs <= 0) return hipSuccess;
    if (dt == 2)
        hipLaunchKernelGGL(k_small_jobs<double>, dim3(n_jobs), dim3(kRedThreads), 0, st, d_jobs, d_ops,
                           (const double *)d_consts, d_out);
    else
        hipLaunchKernelGGL(k_small_jobs<float>, dim3(n_jobs), dim3(kRedThreads), 0, st, d_jobs, d_ops,
                           (const float *)d_consts, d_out);
    return hipGetLastError();
}

}  // namespace sv
