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

#include <cstdint>

#include "sv_kernels.hpp"
#include "sv_plan.hpp"
#include "sv_swizzle.hpp"

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

// ---------------------------------------------------------------------------
// Register-tile operations. P, PA, PB are register-bit positions (compile
// time); every loop is fully unrolled so the tile never leaves VGPRs.

template <int P, typename T, int NR>
__device__ __forceinline__ void r_h(cpx<T> (&a)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        const int j1 = j | (1 << P);
        const cpx<T> x0 = a[j], x1 = a[j1];
        a[j] = cadd(x0, x1);
        a[j1] = csub(x0, x1);
    }
}

template <int P, typename T, int NR>
__device__ __forceinline__ void r_dense1(cpx<T> (&a)[NR], const T *m) {
    const cpx<T> g00 = ldc(m), g01 = ldc(m + 2), g10 = ldc(m + 4), g11 = ldc(m + 6);
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        const int j1 = j | (1 << P);
        const cpx<T> x0 = a[j], x1 = a[j1];
        a[j] = cmul2(g00, x0, g01, x1);
        a[j1] = cmul2(g10, x0, g11, x1);
    }
}

template <int P, typename T, int NR>
__device__ __forceinline__ void r_x(cpx<T> (&a)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        const int j1 = j | (1 << P);
        const cpx<T> t = a[j];
        a[j] = a[j1];
        a[j1] = t;
    }
}

// Y: (x0, x1) -> (-i x1, i x0)
template <int P, typename T, int NR>
__device__ __forceinline__ void r_y(cpx<T> (&a)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        const int j1 = j | (1 << P);
        const cpx<T> x0 = a[j], x1 = a[j1];
        a[j] = mk<T>(x1.y, -x1.x);
        a[j1] = mk<T>(-x0.y, x0.x);
    }
}

// Controlled swap on bit P, control = register bit PC.
template <int P, int PC, typename T, int NR>
__device__ __forceinline__ void r_cx_reg(cpx<T> (&a)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        if (!(j & (1 << PC))) continue;
        const int j1 = j | (1 << P);
        const cpx<T> t = a[j];
        a[j] = a[j1];
        a[j1] = t;
    }
}

// Controlled swap on bit P with a control bit that is the same for every
// register slot of this thread (selects, no divergent branch).
template <int P, typename T, int NR>
__device__ __forceinline__ void r_cx_uni(cpx<T> (&a)[NR], bool c) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (1 << P)) continue;
        const int j1 = j | (1 << P);
        const cpx<T> x0 = a[j], x1 = a[j1];
        a[j] = c ? x1 : x0;
        a[j1] = c ? x0 : x1;
    }
}

// SWAP of register bits PA > PB: exchange slots with (bA, bB) = (1, 0) and (0, 1).
template <int PA, int PB, typename T, int NR>
__device__ __forceinline__ void r_swap(cpx<T> (&a)[NR]) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (!(j & (1 << PA)) || (j & (1 << PB))) continue;
        const int j2 = (j & ~(1 << PA)) | (1 << PB);
        const cpx<T> t = a[j];
        a[j] = a[j2];
        a[j2] = t;
    }
}

// 4x4 on register bits PA (high local bit) > PB (low local bit).
template <int PA, int PB, typename T, int NR>
__device__ __forceinline__ void r_dense2(cpx<T> (&a)[NR], const T *m) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & ((1 << PA) | (1 << PB))) continue;
        const int jj[4] = {j, j | (1 << PB), j | (1 << PA), j | (1 << PA) | (1 << PB)};
        cpx<T> x[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) x[l] = a[jj[l]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const T *row = m + 8 * r;
            cpx<T> acc = cmul2(ldc(row), x[0], ldc(row + 2), x[1]);
            acc = cadd(acc, cmul2(ldc(row + 4), x[2], ldc(row + 6), x[3]));
            a[jj[r]] = acc;
        }
    }
}

// 1-qubit diagonal with the qubit on register bit P.
template <int P, typename T, int NR>
__device__ __forceinline__ void r_d1_reg(cpx<T> (&a)[NR], const T *d) {
    const cpx<T> d0 = ldc(d), d1 = ldc(d + 2);
#pragma unroll
    for (int j = 0; j < NR; ++j) a[j] = cmul(a[j], (j & (1 << P)) ? d1 : d0);
}

// 2-qubit diagonal, both qubits on register bits (PA = q0's bit, PB = q1's).
template <int PA, int PB, typename T, int NR>
__device__ __forceinline__ void r_d2_regreg(cpx<T> (&a)[NR], const T *d) {
    cpx<T> dd[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) dd[l] = ldc(d + 2 * l);
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int l = (((j >> PA) & 1) << 1) | ((j >> PB) & 1);
        a[j] = cmul(a[j], dd[l]);
    }
}

// 2-qubit diagonal: q0 on register bit PA, q1's bit known per thread (ub).
template <int PA, typename T, int NR>
__device__ __forceinline__ void r_d2_reg_hi(cpx<T> (&a)[NR], const T *d, int ub) {
    const cpx<T> e0 = ldc(d + 2 * (0 + ub)), e1 = ldc(d + 2 * (2 + ub));
#pragma unroll
    for (int j = 0; j < NR; ++j) a[j] = cmul(a[j], (j & (1 << PA)) ? e1 : e0);
}
// 2-qubit diagonal: q1 on register bit PB, q0's bit known per thread (ub).
template <int PB, typename T, int NR>
__device__ __forceinline__ void r_d2_reg_lo(cpx<T> (&a)[NR], const T *d, int ub) {
    const cpx<T> e0 = ldc(d + 2 * (2 * ub + 0)), e1 = ldc(d + 2 * (2 * ub + 1));
#pragma unroll
    for (int j = 0; j < NR; ++j) a[j] = cmul(a[j], (j & (1 << PB)) ? e1 : e0);
}

template <typename T, int NR>
__device__ __forceinline__ void r_mul_all(cpx<T> (&a)[NR], cpx<T> d) {
#pragma unroll
    for (int j = 0; j < NR; ++j) a[j] = cmul(a[j], d);
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

// Per-layout index tables of one thread.
template <int NR>
struct LayoutIdx {
    uint64_t gthr;        // global index bits contributed by the thread bits
    uint64_t greg[NR];    // ... by the register slot bits
    uint32_t sthr;        // swizzled LDS slot, thread part
    uint32_t sreg[NR];    // ... register part
};

template <int R, int M>
__device__ __forceinline__ void make_layout(LayoutIdx<1 << R> &L, const DevLayout &dl,
                                            const uint8_t *q, int w, int tid) {
    constexpr int NR = 1 << R;
    uint64_t g = 0;
    uint32_t l = 0;
    for (int s = 0; s < w; ++s) {
        if ((tid >> s) & 1) {
            const int lb = dl.thr_local[s];
            l |= 1u << lb;
            g |= 1ull << q[lb];
        }
    }
    L.gthr = g;
    L.sthr = l ^ swz_fold(l, M);
    uint64_t gb[R];
    uint32_t lbit[R];
#pragma unroll
    for (int p = 0; p < R; ++p) {
        lbit[p] = 1u << dl.reg_local[p];
        gb[p] = 1ull << q[dl.reg_local[p]];
    }
    L.greg[0] = 0;
    uint32_t lr[NR];
    lr[0] = 0;
#pragma unroll
    for (int j = 1; j < NR; ++j) {
        const int p = __builtin_ctz(j);
        L.greg[j] = L.greg[j & (j - 1)] | gb[p];
        lr[j] = lr[j & (j - 1)] | lbit[p];
    }
#pragma unroll
    for (int j = 0; j < NR; ++j) L.sreg[j] = lr[j] ^ swz_fold(lr[j], M);
}

template <typename T>
struct PassTraits;
template <>
struct PassTraits<double> {
    static constexpr int R = kRegBitsC128;
    static constexpr int M = 3;
};
template <>
struct PassTraits<float> {
    static constexpr int R = kRegBitsC64;
    static constexpr int M = 4;
};

template <typename T>
__global__ __launch_bounds__(256) void k_pass(cpx<T> *__restrict__ state, uint64_t n_amps,
                                              const DevPass *__restrict__ passes, int pass_idx,
                                              const DevLayout *__restrict__ layouts,
                                              const DevOp *__restrict__ ops,
                                              const T *__restrict__ consts,
                                              uint64_t const_stride) {
    constexpr int R = PassTraits<T>::R;
    constexpr int M = PassTraits<T>::M;
    constexpr int NR = 1 << R;
    __shared__ cpx<T> lds[NR << kMaxThreadBits];

    const DevPass &P = passes[pass_idx];
    const int tid = threadIdx.x;
    const int w = P.w;
    const int k = P.k;
    uint8_t q[32];
#pragma unroll
    for (int l = 0; l < 32; ++l) q[l] = P.q[l];

    cpx<T> *st = state + (uint64_t)blockIdx.y * n_amps;
    const T *cst = consts + (uint64_t)blockIdx.y * const_stride;

    // Global index of the tile's amplitude with all tile-local bits zero:
    // the tile number with zeros inserted at the tile qubits (ascending).
    uint64_t base = blockIdx.x;
    for (int l = 0; l < k; ++l) {
        const int b = q[l];
        base = ((base >> b) << (b + 1)) | (base & ((1ull << b) - 1));
    }

    LayoutIdx<NR> L;
    int cur = P.layout_begin;
    make_layout<R, M>(L, layouts[cur], q, w, tid);

    cpx<T> a[NR];
    const bool pair_io = (sizeof(T) == 4) && layouts[cur].reg_local[0] == 0 && q[0] == 0;
    if (P.flags & PASS_GENERATE) {
        // On-demand Hadamard-layer amplitudes of H^M |j>:
        // 2^(-|M|/2) (-1)^popcount(i & j & M) where i agrees with j off M.
        const uint64_t gm = P.gen_mask, gj = P.gen_j;
        const T mag = (T)P.gen_scale;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const uint64_t i = base | L.gthr | L.greg[j];
            const bool on = ((i ^ gj) & ~gm) == 0;
            const T v = (__popcll(i & gj & gm) & 1) ? -mag : mag;
            a[j] = mk<T>(on ? v : (T)0, (T)0);
        }
    } else if (pair_io) {
#pragma unroll
        for (int j = 0; j < NR; j += 2) {
            const float4 v = *reinterpret_cast<const float4 *>(st + (base | L.gthr | L.greg[j]));
            a[j] = mk<T>((T)v.x, (T)v.y);
            a[j + 1] = mk<T>((T)v.z, (T)v.w);
        }
    } else {
#pragma unroll
        for (int j = 0; j < NR; ++j) a[j] = st[base | L.gthr | L.greg[j]];
    }

    for (int oi = P.op_begin; oi < P.op_end; ++oi) {
        const DevOp op = ops[oi];
        switch (op.code) {
        case OP_EXCH: {
            __syncthreads();
#pragma unroll
            for (int j = 0; j < NR; ++j) lds[L.sthr ^ L.sreg[j]] = a[j];
            __syncthreads();
            cur = P.layout_begin + op.a;
            make_layout<R, M>(L, layouts[cur], q, w, tid);
#pragma unroll
            for (int j = 0; j < NR; ++j) a[j] = lds[L.sthr ^ L.sreg[j]];
            break;
        }
        case OP_D1: {
            const T *d = cst + op.data;
            const int kind = op.sa & ~SRC_POS_MASK, pos = op.sa & SRC_POS_MASK;
            if (kind == SRC_REG) {
                SV_SWITCH_A(pos, r_d1_reg<PA>(a, d))
            } else {
                const int bit = kind == SRC_THR ? (tid >> pos) & 1 : (int)((base >> pos) & 1);
                r_mul_all(a, ldc(d + 2 * bit));
            }
            break;
        }
        case OP_D2: {
            const T *d = cst + op.data;
            const int ka = op.sa & ~SRC_POS_MASK, pa = op.sa & SRC_POS_MASK;
            const int kb = op.sb & ~SRC_POS_MASK, pb = op.sb & SRC_POS_MASK;
            const int ua = ka == SRC_THR ? (tid >> pa) & 1 : (int)((base >> pa) & 1);
            const int ub = kb == SRC_THR ? (tid >> pb) & 1 : (int)((base >> pb) & 1);
            if (ka == SRC_REG && kb == SRC_REG) {
                SV_SWITCH_A(pa, SV_SWITCH_B(pb, if constexpr (PA != PB) r_d2_regreg<PA, PB>(a, d)))
            } else if (ka == SRC_REG) {
                SV_SWITCH_A(pa, r_d2_reg_hi<PA>(a, d, ub))
            } else if (kb == SRC_REG) {
                SV_SWITCH_B(pb, r_d2_reg_lo<PB>(a, d, ua))
            } else {
                r_mul_all(a, ldc(d + 2 * ((ua << 1) | ub)));
            }
            break;
        }
        case OP_MARK: {
            if (base == op.data && tid == (int)op.b) {
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    if (j == (int)op.a) a[j] = mk<T>(-a[j].x, -a[j].y);
            }
            break;
        }
        case OP_DENSE1: {
            const T *m = cst + op.data;
            SV_SWITCH_A(op.a, r_dense1<PA>(a, m))
            break;
        }
        case OP_H: {
            SV_SWITCH_A(op.a, r_h<PA>(a))
            break;
        }
        case OP_X: {
            SV_SWITCH_A(op.a, r_x<PA>(a))
            break;
        }
        case OP_Y: {
            SV_SWITCH_A(op.a, r_y<PA>(a))
            break;
        }
        case OP_CX: {
            const int kc = op.sa & ~SRC_POS_MASK, pc = op.sa & SRC_POS_MASK;
            if (kc == SRC_REG) {
                SV_SWITCH_A(op.a, SV_SWITCH_B(pc, if constexpr (PA != PB) r_cx_reg<PA, PB>(a)))
            } else {
                const bool c = kc == SRC_THR ? ((tid >> pc) & 1) : ((base >> pc) & 1);
                SV_SWITCH_A(op.a, r_cx_uni<PA>(a, c))
            }
            break;
        }
        case OP_SWAP: {
            SV_SWITCH_A(op.a, SV_SWITCH_B(op.b, if constexpr (PA > PB) r_swap<PA, PB>(a)))
            break;
        }
        case OP_DENSE2: {
            const T *m = cst + op.data;
            SV_SWITCH_A(op.a, SV_SWITCH_B(op.b, if constexpr (PA > PB) r_dense2<PA, PB>(a, m)))
            break;
        }
        case OP_SCALE: {
            r_scale(a, cst[op.data]);
            break;
        }
        default:
            break;
        }
    }

    const bool pair_out = (sizeof(T) == 4) && layouts[cur].reg_local[0] == 0 && q[0] == 0;
    if (pair_out) {
#pragma unroll
        for (int j = 0; j < NR; j += 2) {
            float4 v;
            v.x = (float)a[j].x;
            v.y = (float)a[j].y;
            v.z = (float)a[j + 1].x;
            v.w = (float)a[j + 1].y;
            *reinterpret_cast<float4 *>(st + (base | L.gthr | L.greg[j])) = v;
        }
    } else {
#pragma unroll
        for (int j = 0; j < NR; ++j) st[base | L.gthr | L.greg[j]] = a[j];
    }
}

// ---------------------------------------------------------------------------
// Whole state in one workgroup's LDS; one operation at a time.

__device__ __forceinline__ uint32_t ins0(uint32_t x, int q) {
    return ((x >> q) << (q + 1)) | (x & ((1u << q) - 1));
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
    for (uint32_t i = tid; i < N; i += nt) s[i] = st[i];
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
        const uint64_t r = i % n_amps;
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

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_reduce_partial(const cpx<T> *__restrict__ state,
                                                                uint64_t n_amps, uint64_t chunk,
                                                                int qubit, double *__restrict__ part,
                                                                int nblk) {
    __shared__ double sh[kRedThreads];
    const cpx<T> *st = state + (uint64_t)blockIdx.y * n_amps;
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    double acc = 0.0;
    for (uint64_t i = lo + threadIdx.x; i < lo + chunk; i += kRedThreads) {
        const cpx<T> v = st[i];
        const double re = (double)v.x, im = (double)v.y;
        const double p = re * re + im * im;
        acc += (qubit >= 0 && ((i >> qubit) & 1)) ? -p : p;
    }
    const double s = block_tree_sum(acc, sh);
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

hipError_t launch_pass(int dt, void *state, uint64_t n_amps, int batch, const DevPass *d_passes,
                       int pass_idx, const DevPass &h_pass, const DevLayout *d_layouts,
                       const DevOp *d_ops, const void *d_consts, uint64_t const_stride,
                       hipStream_t st) {
    const dim3 grid((unsigned)h_pass.tiles, (unsigned)batch);
    const dim3 block(1u << h_pass.w);
    if (dt == 2)
        hipLaunchKernelGGL(k_pass<double>, grid, block, 0, st, (cpx<double> *)state, n_amps,
                           d_passes, pass_idx, d_layouts, d_ops, (const double *)d_consts,
                           const_stride);
    else
        hipLaunchKernelGGL(k_pass<float>, grid, block, 0, st, (cpx<float> *)state, n_amps,
                           d_passes, pass_idx, d_layouts, d_ops, (const float *)d_consts,
                           const_stride);
    return hipGetLastError();
}

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
static int reduce_blocks(int n) {
    if (n <= 12) return 1;
    const int b = n - 12;               // chunks of 4096 amplitudes ...
    return 1 << (b < 10 ? b : 10);      // ... at most 1024 blocks
}

size_t reduce_partials_size(int n) { return (size_t)reduce_blocks(n); }

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

}  // namespace sv
