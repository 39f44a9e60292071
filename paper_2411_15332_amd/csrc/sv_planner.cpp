// Gate classification, pass planning and operation payloads (host side).
//
// Classification follows the paper's observation (Sec. II-C, Table 1) that
// most gates are sparse. Diagonal gates are applied from their phases alone,
// monomial gates from their gate-local (value, index) form — the DAX entry of
// Sec. III-A1 restricted to the gate's own 2^k x 2^k matrix — and a
// Hadamard from one magnitude plus index-derived signs (RH, Sec. III-B1).
// Where the paper composes a stage's gates into one compressed operator before
// a single matrix-vector product (Sec. III-A2, MTP before MVM), the planner
// composes a run of gates into one pass over HBM: permutations are absorbed
// into the tile's addressing (the index part of a DAX entry), runs of 1-qubit
// gates on one register bit are multiplied into one 2x2, and diagonal factors
// that are constant across a thread's registers are folded into one scalar.
// The 2^n x 2^n operator is never formed.
#include "sv_planner.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <stdexcept>

#include "sv_swizzle.hpp"

namespace sv {

using cd = std::complex<double>;

static inline int popc(uint64_t x) { return __builtin_popcountll(x); }
static inline uint64_t bit(int q) { return 1ull << q; }

static bool is_angled(int kind) {
    return kind == SV_GATE_RX || kind == SV_GATE_RY || kind == SV_GATE_RZ ||
           kind == SV_GATE_P || kind == SV_GATE_CPHASE || kind == SV_GATE_CRZ ||
           kind == SV_GATE_RZZ || kind == SV_GATE_CU1 || kind == SV_GATE_RXX ||
           kind == SV_GATE_RYY || kind == SV_GATE_RZX;
}
static bool is_2q(int kind) {
    switch (kind) {
    case SV_GATE_CNOT: case SV_GATE_CZ: case SV_GATE_SWAP: case SV_GATE_CPHASE: case SV_GATE_U2:
    case SV_GATE_CY: case SV_GATE_ISWAP: case SV_GATE_DCX: case SV_GATE_CRZ: case SV_GATE_RZZ:
    case SV_GATE_CU1: case SV_GATE_RXX: case SV_GATE_RYY: case SV_GATE_RZX: case SV_GATE_ECR:
    case SV_GATE_CH: case SV_GATE_CSX: case SV_GATE_CU3: case SV_GATE_CU:
        return true;
    default:
        return false;
    }
}
// Angles a several-angle gate reads from the parameter table (0: none).
static size_t multi_angles(int kind) {
    switch (kind) {
    case SV_GATE_R: return 2;
    case SV_GATE_U: case SV_GATE_CU3: return 3;
    case SV_GATE_CU: return 4;
    default: return 0;
    }
}
static bool is_3q(int kind) { return kind == SV_GATE_CCX || kind == SV_GATE_CSWAP; }
// Reals a matrix gate reads from the parameter table (0: not a matrix gate).
static size_t matrix_reals(int kind) {
    return kind == SV_GATE_U1 ? 8 : kind == SV_GATE_U2 ? 32 : 0;
}

bool validate_gates(int n, const sv_gate *gates, size_t n_gates, size_t n_params,
                    bool params_given, std::string &err) {
    const uint64_t N = 1ull << n;
    for (size_t i = 0; i < n_gates; ++i) {
        const sv_gate &g = gates[i];
        char buf[160];
        if (g.kind < 0 || g.kind >= SV_GATE_KIND_COUNT) {
            snprintf(buf, sizeof buf, "gate %zu: unknown kind %d", i, g.kind);
            err = buf;
            return false;
        }
        if (g.kind == SV_GATE_MARK) {
            if (g.index >= N) {
                snprintf(buf, sizeof buf, "gate %zu: MARK index %llu >= 2^%d", i,
                         (unsigned long long)g.index, n);
                err = buf;
                return false;
            }
        } else if (is_3q(g.kind)) {
            const int64_t q2 = (int64_t)g.index;
            if (g.q0 < 0 || g.q0 >= n || g.q1 < 0 || g.q1 >= n || g.index >= (uint64_t)n ||
                g.q0 == g.q1 || g.q0 == q2 || g.q1 == q2) {
                snprintf(buf, sizeof buf, "gate %zu: qubits (%d, %d, %lld) invalid for n = %d", i,
                         g.q0, g.q1, (long long)q2, n);
                err = buf;
                return false;
            }
        } else if (is_2q(g.kind)) {
            if (g.q0 < 0 || g.q0 >= n || g.q1 < 0 || g.q1 >= n || g.q0 == g.q1) {
                snprintf(buf, sizeof buf, "gate %zu: qubits (%d, %d) invalid for n = %d", i,
                         g.q0, g.q1, n);
                err = buf;
                return false;
            }
        } else if (g.q0 < 0 || g.q0 >= n) {
            snprintf(buf, sizeof buf, "gate %zu: qubit %d out of range for n = %d", i, g.q0, n);
            err = buf;
            return false;
        }
        if (matrix_reals(g.kind)) {
            if (g.param < 0 || !params_given || (size_t)g.param + matrix_reals(g.kind) > n_params) {
                snprintf(buf, sizeof buf,
                         "gate %zu: U%d needs %zu matrix reals from parameter %d (n_params = %zu)",
                         i, g.kind == SV_GATE_U1 ? 1 : 2, matrix_reals(g.kind), g.param, n_params);
                err = buf;
                return false;
            }
        } else if (multi_angles(g.kind)) {
            if (g.param < 0 || !params_given || (size_t)g.param + multi_angles(g.kind) > n_params) {
                snprintf(buf, sizeof buf, "gate %zu: kind %d needs %zu angles from parameter %d (n_params = %zu)",
                         i, g.kind, multi_angles(g.kind), g.param, n_params);
                err = buf;
                return false;
            }
        } else if (g.param >= 0) {
            if (!is_angled(g.kind)) {
                snprintf(buf, sizeof buf, "gate %zu: kind %d takes no parameter", i, g.kind);
                err = buf;
                return false;
            }
            if (!params_given || (size_t)g.param >= n_params) {
                snprintf(buf, sizeof buf, "gate %zu: parameter %d not supplied (n_params = %zu)",
                         i, g.param, n_params);
                err = buf;
                return false;
            }
        } else if (g.param < -1) {
            snprintf(buf, sizeof buf, "gate %zu: param %d invalid", i, g.param);
            err = buf;
            return false;
        } else if (is_angled(g.kind) && !std::isfinite(g.angle)) {
            snprintf(buf, sizeof buf, "gate %zu: angle is not finite", i);
            err = buf;
            return false;
        }
    }
    return true;
}

CGate classify(const sv_gate &g, int n, int src) {
    CGate c;
    c.src = src;
    c.q0 = g.q0;
    c.q1 = g.q1;
    switch (g.kind) {
    case SV_GATE_I: c.cls = G_NOP; break;
    case SV_GATE_X: c.cls = G_X; break;
    case SV_GATE_Y: c.cls = G_Y; break;
    case SV_GATE_Z: case SV_GATE_S: case SV_GATE_SDG: case SV_GATE_T: case SV_GATE_TDG:
    case SV_GATE_RZ: case SV_GATE_P:
        c.cls = G_D1; break;
    case SV_GATE_H: c.cls = G_H; break;
    case SV_GATE_RX: case SV_GATE_RY: case SV_GATE_U1: c.cls = G_DENSE1; break;
    case SV_GATE_U2: c.cls = G_DENSE2; break;
    case SV_GATE_CNOT: c.cls = G_CX; break;
    case SV_GATE_CZ: case SV_GATE_CPHASE: c.cls = G_D2; break;
    case SV_GATE_SWAP: c.cls = G_SWAP; break;
    case SV_GATE_MARK: c.cls = G_MARK; c.index = g.index; break;
    case SV_GATE_CCX: c.cls = G_CCX; c.q2 = (int)g.index; break;
    default:
        // the composite kinds (CY ... CSWAP) are lowered before planning
        if (g.kind >= SV_GATE_CY) throw std::logic_error("gate kind reached the planner unlowered");
        c.cls = G_NOP;
        break;
    }
    switch (c.cls) {
    case G_D1: c.diag = true; c.support = bit(c.q0); break;
    case G_D2: c.diag = true; c.support = bit(c.q0) | bit(c.q1); break;
    case G_MARK: c.diag = true; c.support = (n >= 64) ? ~0ull : (bit(n) - 1); break;
    // X and Y on a qubit outside the tile flip a bit of the global XOR
    // translation of addresses (no data moves), so they need no tile slot
    case G_X: case G_Y: c.support = bit(c.q0); break;
    case G_H: case G_DENSE1: c.support = c.qneed = c.rneed = bit(c.q0); break;
    case G_CX: c.support = bit(c.q0) | bit(c.q1); c.qneed = c.rneed = bit(c.q1); break;
    case G_SWAP: c.support = c.qneed = bit(c.q0) | bit(c.q1); break;
    case G_DENSE2: c.support = c.qneed = c.rneed = bit(c.q0) | bit(c.q1); break;
    case G_CCX: c.support = bit(c.q0) | bit(c.q1) | bit(c.q2); c.qneed = c.rneed = bit(c.q2); break;
    default: break;
    }
    return c;
}

bool tile_geometry(int n, const PlanOptions &opt, int &k, int &w) {
    k = std::min(n, opt.w_max + opt.R);
    w = k - opt.R;
    return w >= 6;
}

// Blocked-qubit bookkeeping for moving a gate past deferred ones: two gates
// commute when both are diagonal or when their supports are disjoint.
struct Blocker {
    uint64_t any = 0, nondiag = 0;
    bool conflicts(const CGate &g) const {
        return g.diag ? (g.support & nondiag) != 0 : (g.support & any) != 0;
    }
    void defer(const CGate &g) {
        any |= g.support;
        if (!g.diag) nondiag |= g.support;
    }
};

// Gates not yet placed, in order: `head` holds gates a pass scanned and
// deferred, followed by order[tail..] (never scanned). A pass stops scanning
// once every qubit is blocked, so a long circuit is not rescanned per pass.
struct GateQueue {
    std::vector<int> head;
    const std::vector<int> *order = nullptr;
    size_t tail = 0;
    bool empty() const { return head.empty() && tail >= order->size(); }
};

// One pass: take gates in order (moving a gate past deferred ones only where
// they commute) while the union of their tile needs fits k qubits, starting
// from the physical bits every tile holds (`low`). Tile sets are physical
// bits: ph / lg map logical qubits to physical bits and back, and a taken
// SWAP that is not inside the tile exchanges its qubits' bits (a relabel:
// the data stays where it is). Returns the tile set; ph / lg end as the map
// after the taken gates. With `commit`, the taken gates go to `taken` and
// `pend` keeps the rest; without, `pend` is left unchanged (a look-ahead).
static uint64_t form_one_pass(const std::vector<CGate> &cg, GateQueue &pend, int n, int k,
                              const PlanOptions &opt, uint64_t low, bool commit,
                              std::vector<int> &taken, std::vector<int> &ph, std::vector<int> &lg) {
    const uint64_t all = (n >= 64) ? ~0ull : (bit(n) - 1);
    uint64_t Q = low & all;
    Blocker blk;
    int dense = 0;
    bool closed = false;
    std::vector<int> new_head;
    auto need_of = [&](uint64_t qm) {
        uint64_t r = 0;
        for (; qm; qm &= qm - 1) r |= bit(ph[__builtin_ctzll(qm)]);
        return r;
    };
    auto visit = [&](int gi) {
        const CGate &g = cg[gi];
        bool take = false;
        if (!blk.conflicts(g)) {
            const bool dense_ok = g.cls != G_DENSE1 || dense < opt.max_dense;
            const uint64_t need = need_of(g.qneed);
            if (dense_ok && (need & ~Q) == 0) take = true;
            else if (dense_ok && popc(Q | need) <= k) { Q |= need; take = true; }
        }
        if (take) {
            if (commit) taken.push_back(gi);
            if (g.cls == G_DENSE1) ++dense;
            if (g.cls == G_SWAP && g.qneed == 0) {
                const int pa = ph[g.q0], pb = ph[g.q1];
                if (!(((Q >> pa) & 1) && ((Q >> pb) & 1))) {
                    std::swap(ph[g.q0], ph[g.q1]);
                    lg[pa] = g.q1;
                    lg[pb] = g.q0;
                }
            }
            if (!opt.fuse) closed = true;
        } else {
            if (commit) new_head.push_back(gi);
            blk.defer(g);
            if ((blk.nondiag & all) == all) closed = true;  // nothing can move past
        }
    };
    size_t hi = 0;
    for (; hi < pend.head.size() && !closed; ++hi) visit(pend.head[hi]);
    size_t t = pend.tail;
    for (; t < pend.order->size() && !closed; ++t) visit((*pend.order)[t]);
    if (commit) {
        // unscanned head entries stay, in order, after the newly deferred ones
        for (; hi < pend.head.size(); ++hi) new_head.push_back(pend.head[hi]);
        pend.head.swap(new_head);
        pend.tail = t;
    }
    return Q;
}

static double hadamard_magnitude(int h) {
    // 2^(-h/2): exact for even h, one rounding of 1/sqrt(2) for odd h
    double s = std::ldexp(1.0, -(h / 2));
    if (h & 1) s *= 0.70710678118654752440;
    return s;
}

namespace {

// Structural class of a pending register-bit product.
enum : uint8_t { PC_I = 0, PC_D, PC_A, PC_H, PC_G };

uint8_t compose_class(uint8_t cur, uint8_t fc) {
    if (cur == PC_I) return fc;
    if ((cur == PC_D || cur == PC_A) && (fc == PC_D || fc == PC_A))
        return cur == fc ? PC_D : PC_A;
    return PC_G;
}

struct Pending {
    uint8_t cls = PC_I;
    bool pure_x = true;
    std::vector<Factor> f;
};

struct Src {
    uint8_t code;   // SRC_* | position
    int inv;        // 1 when the physical bit is the label bit XOR 1
    bool reg;
    int p;          // register bit when reg
};

struct PassCtx {
    const PlanOptions &opt;
    Plan &P;
    const std::vector<CGate> &cg;
    int n, k, w;
    uint8_t q[32];          // physical bit position of label l (ascending): the tile's bits
    uint8_t gpos[32];       // physical bit each label is addressed at by the layout being built
    // Physical bit of every logical qubit off the tile (ph) and the logical
    // qubit at every physical bit off the tile (lg); SWAPs that leave the
    // tile change them during the pass. label_logi: logical qubit of every
    // tile label (label_of is its inverse, -1 off the tile).
    std::vector<int> ph, lg;
    int label_logi[32];
    // Global XOR translation: physical address a holds the amplitude of
    // (remapped) index a ^ gx. The load layout's addresses carry all of
    // gx_start, every later layout's its bits off the tile (a workgroup
    // stores in place, to the addresses it loaded, with the tile's own bits
    // canonical). X / Y on a qubit off the tile flips its bit in gxd: the
    // tile base the ops see (the kernel's `base`, the logical base at the
    // pass's start) then differs from the data's by gxd, which the tile
    // sources take as an inversion.
    uint64_t gx_start = 0, gx_off = 0, gxd = 0;
    uint64_t addr_xor = 0;          // physical address XOR of the next layout record
    int label_of[64];
    // layout state: position of every label and the XOR mask
    int reg_label[kLayoutRegBits], thr_label[kLayoutThreadBits];
    int pos_reg[32], pos_thr[32];   // register / thread bit holding label l, or -1
    uint32_t xmask = 0;
    int layout_begin = 0;
    int cur_layout = -1;            // pass-relative index of the materialized state, -1: not yet
    Pending pend[kLayoutRegBits];
    bool f_used = false;
    int op_floor = 0;   // first op of the current pass (records never merge across passes)
    int h_count = 0;
    int first_payload = -1;
    // Pending uniform diagonals (thread / tile-base bits), merged into one
    // OP_UDN emitted before the next operation that consumes f.
    std::vector<UContrib> ud;
    std::vector<uint16_t> uterm;   // (s1 | s2 << 8)

    PassCtx(const PlanOptions &o, Plan &p, const std::vector<CGate> &g, int n_, int k_, int w_)
        : opt(o), P(p), cg(g), n(n_), k(k_), w(w_) {}

    uint64_t U_labels() const {   // labels that may hold registers in a storable layout
        uint64_t u = 0;
        for (int l = opt.v + 6; l < k; ++l) u |= bit(l);
        return u;
    }

    // A layout state: the label of every register and thread bit, and the
    // XOR mask. `fixed_thr`: thread bits below it are pinned by the layout's
    // kind (lanes of a storable layout hold labels v..v+5; the first m lanes of
    // a general layout hold labels with independent swizzle images).
    struct LState {
        int reg[kLayoutRegBits];
        int thr[kLayoutThreadBits];
        uint32_t xmask;
        int fixed_thr;
        bool storable;
    };

    LState save() const {
        LState st{};
        for (int p = 0; p < opt.R; ++p) st.reg[p] = reg_label[p];
        for (int t = 0; t < w; ++t) st.thr[t] = thr_label[t];
        st.xmask = xmask;
        st.fixed_thr = w;
        st.storable = false;
        return st;
    }

    void load(const LState &st) {
        for (int l = 0; l < 32; ++l) pos_reg[l] = pos_thr[l] = -1;
        for (int p = 0; p < opt.R; ++p) { reg_label[p] = st.reg[p]; pos_reg[st.reg[p]] = p; }
        for (int t = 0; t < w; ++t) { thr_label[t] = st.thr[t]; pos_thr[st.thr[t]] = t; }
        xmask = st.xmask;
        cur_layout = -1;
    }

    // regs_u: R - v labels from U_labels(); lanes hold labels v..v+5.
    LState storable(uint64_t regs_u) const {
        LState st{};
        int p = 0, t = 0;
        for (int l = 0; l < opt.v; ++l) st.reg[p++] = l;
        for (int l = 0; l < k; ++l) if ((regs_u >> l) & 1) st.reg[p++] = l;
        for (int l = opt.v; l < opt.v + 6; ++l) st.thr[t++] = l;
        const uint64_t rest = U_labels() & ~regs_u;
        for (int l = 0; l < k; ++l) if ((rest >> l) & 1) st.thr[t++] = l;
        st.xmask = 0;
        st.fixed_thr = 6;
        st.storable = true;
        return st;
    }

    // regs: R labels; lanes 0..m-1 get labels whose swizzle images are
    // linearly independent (conflict-free LDS rows).
    LState general(uint64_t regs) const {
        LState st{};
        int p = 0;
        for (int l = 0; l < k; ++l) if ((regs >> l) & 1) st.reg[p++] = l;
        std::vector<int> lanes, others;
        uint32_t basis[8] = {0};
        for (int l = 0; l < k; ++l) {
            if ((regs >> l) & 1) continue;
            uint32_t x = swz_image(l, opt.m);
            for (int b = opt.m - 1; b >= 0 && x; --b) {
                if (!((x >> b) & 1)) continue;
                if (basis[b]) x ^= basis[b];
                else { basis[b] = x; break; }
            }
            if (x && (int)lanes.size() < opt.m) lanes.push_back(l);
            else others.push_back(l);
        }
        int t = 0;
        for (int l : lanes) st.thr[t++] = l;
        for (int l : others) st.thr[t++] = l;
        st.xmask = 0;
        st.fixed_thr = opt.m;
        st.storable = false;
        return st;
    }

    static int find_in(const int *arr, int cnt, int l) {
        for (int i = 0; i < cnt; ++i) if (arr[i] == l) return i;
        return -1;
    }

    // Register position p of state b may be re-assigned (a storable complex64
    // layout keeps label 0 in register 0 for its paired 16-byte accesses).
    bool reg_free(const LState &b, int p) const { return !(b.storable && opt.v && p == 0); }

    // Half-tile exchange from a to b: find a label l >= m (its LDS slot bit is
    // outside the swizzle bits, so dropping it keeps slots distinct and
    // conflict-free) held at the same register position, or failing that the
    // same thread bit, in both layouts. b may be permuted to make that true and
    // takes a's XOR bit of l. Returns the split source and label.
    bool find_split(const LState &a, LState &b, uint8_t &src, int &lab) const {
        for (int p = 0; p < opt.R; ++p) {
            const int l = a.reg[p];
            if (l < opt.m) continue;
            const int pb = find_in(b.reg, opt.R, l);
            if (pb < 0) continue;
            if (pb != p) {
                if (!reg_free(b, p) || !reg_free(b, pb)) continue;
                std::swap(b.reg[p], b.reg[pb]);
            }
            b.xmask = (b.xmask & ~(1u << l)) | (a.xmask & (1u << l));
            src = (uint8_t)(SRC_REG | p);
            lab = l;
            return true;
        }
        for (int t = w - 1; t >= 0; --t) {   // high thread bits first: whole waves per half
            const int l = a.thr[t];
            if (l < opt.m) continue;
            const int tb = find_in(b.thr, w, l);
            if (tb < 0) continue;
            if (tb != t) {
                if (t < b.fixed_thr || tb < b.fixed_thr) continue;
                std::swap(b.thr[t], b.thr[tb]);
            }
            b.xmask = (b.xmask & ~(1u << l)) | (a.xmask & (1u << l));
            src = (uint8_t)(SRC_THR | t);
            lab = l;
            return true;
        }
        return false;
    }

    void emit_exch(int wl, int rl, uint8_t src, int lab) {
        HostOp &ex = emit(OP_EXCH);
        ex.hdr.a = (uint8_t)wl;
        ex.hdr.b = (uint8_t)rl;
        ex.hdr.sa = src;
        ex.hdr.sb = (uint8_t)lab;
        ++P.n_exch;
    }

    // Re-distribute the tile (pending register products already flushed) from
    // the current layout into b. When no label can split the exchange, go
    // through an intermediate layout M: b with one of a's register labels
    // l >= m moved into the register position it has in a (R > m guarantees
    // one). a -> M splits on that register; M -> b splits on a register or
    // thread position the two share (all but one or two of them).
    void exchange_to(LState b) {
        const LState a = save();
        const int wl = layout_index();
        uint8_t src = 0;
        int lab = -1;
        if (find_split(a, b, src, lab)) {
            load(b);
            emit_exch(wl, layout_index(), src, lab);
            return;
        }
        int pk = -1;
        for (int p = 0; p < opt.R; ++p)
            if (a.reg[p] >= opt.m) { pk = p; break; }
        LState M = b;
        M.storable = false;
        M.fixed_thr = w;
        int keep = -1;
        if (pk >= 0) {
            // M: b with a's register label `keep` at its register position in a
            keep = a.reg[pk];
            const int pb = find_in(b.reg, opt.R, keep);
            if (pb >= 0) {
                std::swap(M.reg[pk], M.reg[pb]);
            } else {
                const int tk = find_in(b.thr, w, keep);
                M.thr[tk] = b.reg[pk];
                M.reg[pk] = keep;
            }
        } else {
            // every register label of a is below m: M is b with one of a's
            // thread labels >= m at its thread position in a
            int tk = -1;
            for (int t = w - 1; t >= 0 && tk < 0; --t)
                if (a.thr[t] >= opt.m) tk = t;
            if (tk < 0) throw std::logic_error("layout exchange: no label to split on");
            keep = a.thr[tk];
            const int tb = find_in(b.thr, w, keep);
            if (tb >= 0) {
                std::swap(M.thr[tk], M.thr[tb]);
            } else {
                const int pb = find_in(b.reg, opt.R, keep);
                M.reg[pb] = b.thr[tk];
                M.thr[tk] = keep;
            }
        }
        M.xmask = a.xmask & (1u << keep);
        uint8_t s1 = 0, s2 = 0;
        int l1 = -1, l2 = -1;
        if (!find_split(a, M, s1, l1)) throw std::logic_error("layout exchange via M: first half");
        load(M);
        const int ml = layout_index();
        emit_exch(wl, ml, s1, l1);
        const LState m2 = save();
        if (!find_split(m2, b, s2, l2)) throw std::logic_error("layout exchange via M: second half");
        load(b);
        emit_exch(ml, layout_index(), s2, l2);
    }

    // Bring the final layout into lane order for the store: lane s holds
    // label lane[s] and, with v, register 0 holds reg0 (labels the store
    // addresses at the tile's lowest bits). Exchanges only when the current
    // layout differs; other registers stay where they are if possible.
    void settle_lanes(const int *lane, int reg0) {
        bool same = true;
        for (int s = 0; s < 6; ++s) same &= thr_label[s] == lane[s];
        if (opt.v) same &= reg_label[0] == reg0;
        if (same) return;
        LState b{};
        uint32_t placed = 0;
        for (int s = 0; s < 6; ++s) { b.thr[s] = lane[s]; placed |= 1u << lane[s]; }
        int p = 0, t = 6;
        if (opt.v) { b.reg[p++] = reg0; placed |= 1u << reg0; }
        for (int pr = opt.v; pr < opt.R; ++pr)
            if (!((placed >> reg_label[pr]) & 1)) { b.reg[p++] = reg_label[pr]; placed |= 1u << reg_label[pr]; }
        for (int l = 0; l < k; ++l) {
            if ((placed >> l) & 1) continue;
            if (p < opt.R) b.reg[p++] = l;
            else b.thr[t++] = l;
            placed |= 1u << l;
        }
        b.xmask = 0;
        b.fixed_thr = 6;
        b.storable = opt.v != 0;   // keeps register 0 pinned in the exchange search
        exchange_to(b);
    }

    bool is_storable() const {
        for (int s = 0; s < 6; ++s)
            if (thr_label[s] < opt.v || thr_label[s] >= opt.v + 6) return false;
        if (opt.v && (reg_label[0] != 0 || (xmask & 1))) return false;
        return true;
    }

    uint64_t reg_labels() const {
        uint64_t r = 0;
        for (int p = 0; p < opt.R; ++p) r |= bit(reg_label[p]);
        return r;
    }

    static uint32_t slot_lin(int l, int m) {
        return (1u << l) ^ (l >= m ? swz_image(l, m) : 0u);
    }

    int layout_index() {
        if (cur_layout >= 0) return cur_layout;
        DevLayout L;
        std::memset(&L, 0, sizeof L);
        for (int s = 0; s < w; ++s) {
            L.thr_goff[s] = 1ull << gpos[thr_label[s]];
            L.thr_slot[s] = slot_lin(thr_label[s], opt.m);
            L.thr_local[s] = (uint8_t)thr_label[s];
        }
        for (int p = 0; p < opt.R; ++p) {
            L.reg_goff[p] = 1ull << gpos[reg_label[p]];
            L.reg_slot[p] = slot_lin(reg_label[p], opt.m);
            L.reg_local[p] = (uint8_t)reg_label[p];
        }
        for (int l = 0; l < k; ++l) {
            if ((xmask >> l) & 1) {
                if (pos_reg[l] >= 0) L.reg_goff_xor ^= 1ull << gpos[l];
                else L.goff_xor ^= 1ull << gpos[l];
                L.slot_xor ^= slot_lin(l, opt.m);
            }
        }
        L.xor_local = xmask;
        L.reg_goff_xor ^= addr_xor;
        // complex64 16-byte I/O: register bit 0 addresses physical bit 0
        if (opt.v && gpos[reg_label[0]] == 0 && !((xmask >> reg_label[0]) & 1) && !(addr_xor & 1))
            L.flags |= LAYOUT_PAIR_IO;
        P.layouts.push_back(L);
        cur_layout = (int)P.layouts.size() - 1 - layout_begin;
        return cur_layout;
    }

    Src src_of(int qubit) const {
        Src s{};
        const int l = label_of[qubit];
        if (l < 0) {
            s.code = (uint8_t)(SRC_TILE | ph[qubit]);
            s.inv = (int)((gxd >> ph[qubit]) & 1);
            s.reg = false;
            return s;
        }
        s.inv = (int)((xmask >> l) & 1);
        if (pos_reg[l] >= 0) {
            s.code = (uint8_t)(SRC_REG | pos_reg[l]);
            s.reg = true;
            s.p = pos_reg[l];
        } else {
            s.code = (uint8_t)(SRC_THR | pos_thr[l]);
            s.reg = false;
        }
        return s;
    }

    HostOp &emit(uint8_t code) {
        P.ops.emplace_back();
        HostOp &o = P.ops.back();
        o.hdr.code = code;
        return o;
    }
    void note_payload() {
        if (first_payload < 0) first_payload = (int)P.ops.size() - 1;
    }

    void compose(int p, Factor f, uint8_t fc, bool is_x) {
        Pending &pd = pend[p];
        pd.cls = compose_class(pd.cls, fc);
        pd.pure_x = pd.pure_x && is_x;
        pd.f.push_back(f);
    }

    // Which halves of register bit p a pending diagonal product touches:
    // bit 0 = the slots with bit value 0, bit 1 = value 1. Gates with a unit
    // first entry (Z, S, SDG, T, TDG, P) touch one half; X factors in the run
    // swap halves for the factors after them.
    int diag_sides(const Pending &pd) const {
        int sides = 0, flip = 0;
        for (const Factor &f : pd.f) {
            if (f.kind == FK_X) { flip ^= 1; continue; }
            if (f.kind == FK_GATE) {
                const int kd = cg_kind(f.gate);
                if (kd == SV_GATE_I) continue;
                if (kd == SV_GATE_Z || kd == SV_GATE_S || kd == SV_GATE_SDG || kd == SV_GATE_T ||
                    kd == SV_GATE_TDG || kd == SV_GATE_P) {
                    sides |= 1 << (1 ^ (f.conj_x ? 1 : 0) ^ flip);
                    continue;
                }
            }
            sides = 3;
        }
        return sides;
    }

    void flush(int p) {
        Pending &pd = pend[p];
        if (pd.cls == PC_I) { pd = Pending(); return; }
        if (pd.cls == PC_D) {
            const int sides = diag_sides(pd);
            if (sides == 1 || sides == 2) {
                HostOp &o = emit(OP_D1H);
                o.hdr.a = (uint8_t)p;
                o.hdr.b = (uint8_t)(sides == 2 ? 1 : 0);
                o.pk = PK_SIDE;
                o.factors = pd.f;
            } else if (sides == 3) {
                emit_ud();
                HostOp &o = emit(OP_D1R);
                o.hdr.a = (uint8_t)p;
                o.pk = PK_DIAG2;
                o.factors = pd.f;
                note_payload();
                f_used = false;   // the op multiplies by the pending per-thread factor
            }
        } else if (pd.cls == PC_A && pd.pure_x) {
            if (opt.v && reg_label[p] == 0) {   // keeps label 0 unflipped for paired 16-byte I/O
                HostOp &o = emit(OP_X);
                o.hdr.a = (uint8_t)p;
            } else {
                xmask ^= 1u << reg_label[p];     // relabel: no data moves
                cur_layout = -1;
                ++P.n_relabel;
            }
        } else if (pd.cls == PC_H) {
            // joins the preceding Hadamard record when that one is the last
            // op emitted and holds other register bits
            if (!P.ops.empty() && (int)P.ops.size() > op_floor && P.ops.back().hdr.code == OP_H &&
                !((P.ops.back().hdr.a >> p) & 1)) {
                P.ops.back().hdr.a |= (uint8_t)(1u << p);
            } else {
                HostOp &o = emit(OP_H);
                o.hdr.a = (uint8_t)(1u << p);
            }
            ++h_count;
        } else {
            emit_ud();
            uint8_t ri = 0;
            if (ri_form(pd.f, ri)) {
                // half the arithmetic of a general 2x2; a pending per-thread
                // factor stays pending (it is the same for every register
                // slot, so it commutes with register-bit operations)
                HostOp &o = emit(OP_DENSE1RI);
                o.hdr.a = (uint8_t)p;
                o.hdr.b = ri;
                o.pk = PK_MAT2RI;
                o.factors = pd.f;
            } else {
                HostOp &o = emit(OP_DENSE1);
                o.hdr.a = (uint8_t)p;
                o.hdr.b = f_used ? 1 : 0;   // fold the pending per-thread factor
                o.pk = PK_MAT2;
                o.factors = pd.f;
                f_used = false;
            }
            note_payload();
        }
        pd = Pending();
    }

    // Entry classes of a 2x2 as sets of phases: bit 0 real, bit 1 imaginary
    // (0: the entry is zero for every parameter value, 3: complex).
    static uint8_t ph_mul(uint8_t a, uint8_t b) {
        if (!a || !b) return 0;
        uint8_t r = 0;
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q)
                if (((a >> p) & 1) && ((b >> q) & 1)) r |= (uint8_t)(1 << ((p + q) & 1));
        return r;
    }
    void factor_classes(const Factor &f, uint8_t c[4]) const {
        const uint8_t Z = 0, R = 1, I = 2, C = 3;
        auto set = [&](uint8_t a, uint8_t b, uint8_t d, uint8_t e) { c[0] = a; c[1] = b; c[2] = d; c[3] = e; };
        switch (f.kind) {
        case FK_X: set(Z, R, R, Z); break;
        case FK_YDIAG: set(I, Z, Z, I); break;
        case FK_H: set(R, R, R, R); break;
        default:
            switch (cg_kind(f.gate)) {
            case SV_GATE_I: case SV_GATE_Z: set(R, Z, Z, R); break;
            case SV_GATE_X: set(Z, R, R, Z); break;
            case SV_GATE_Y: set(Z, I, I, Z); break;
            case SV_GATE_H: case SV_GATE_RY: set(R, R, R, R); break;
            case SV_GATE_S: case SV_GATE_SDG: set(R, Z, Z, I); break;
            case SV_GATE_T: case SV_GATE_TDG: case SV_GATE_P: set(R, Z, Z, C); break;
            case SV_GATE_RX: set(R, I, I, R); break;
            case SV_GATE_RZ: set(C, Z, Z, C); break;
            default: set(C, C, C, C); break;
            }
        }
        if (f.conj_x) {
            std::swap(c[0], c[3]);
            std::swap(c[1], c[2]);
        }
    }
    // Whether the product of `fs` has, for every parameter value, the form
    // diag(i^g0, i^g1) R diag(1, i^bt) with R real; `flags` = g0 | g1 << 1 | bt << 2.
    bool ri_form(const std::vector<Factor> &fs, uint8_t &flags) const {
        if (!gkinds) return false;
        uint8_t m[4] = {1, 0, 0, 1};
        for (const Factor &f : fs) {
            uint8_t c[4];
            factor_classes(f, c);
            const uint8_t n[4] = {(uint8_t)(ph_mul(c[0], m[0]) | ph_mul(c[1], m[2])),
                                  (uint8_t)(ph_mul(c[0], m[1]) | ph_mul(c[1], m[3])),
                                  (uint8_t)(ph_mul(c[2], m[0]) | ph_mul(c[3], m[2])),
                                  (uint8_t)(ph_mul(c[2], m[1]) | ph_mul(c[3], m[3]))};
            std::copy(n, n + 4, m);
        }
        for (int fl = 0; fl < 8; ++fl) {
            bool ok = true;
            for (int e = 0; e < 4 && ok; ++e) {
                const int r = e >> 1, col = e & 1;
                const int ph = (((fl >> r) & 1) + (col ? (fl >> 2) & 1 : 0)) & 1;
                ok = m[e] == 0 || m[e] == (uint8_t)(1 << ph);
            }
            if (ok) {
                flags = (uint8_t)fl;
                return true;
            }
        }
        return false;
    }
    void flush_nondiag(int p) {
        if (pend[p].cls != PC_I && pend[p].cls != PC_D) flush(p);
    }
    void flush_all() {
        for (int p = 0; p < opt.R; ++p) flush(p);
        emit_ud();
        if (f_used) {
            emit(OP_APPLYF);
            f_used = false;
        }
    }

    int cg_kind(int src) const { return gkinds ? gkinds[src] : -1; }
    const int *gkinds = nullptr;   // sv_gate kind of every source gate

    // Term slot of the pending OP_UDN for the bit of s1 (s2 = kNoSource) or
    // the AND of two bits; -1 when the operation is full.
    int term_slot(uint8_t s1, uint8_t s2) {
        if (s2 != kNoSource && s2 < s1) std::swap(s1, s2);
        const uint16_t key = (uint16_t)(s1 | (s2 << 8));
        for (size_t i = 0; i < uterm.size(); ++i) if (uterm[i] == key) return (int)i;
        if ((int)uterm.size() >= opt.ud_max) return -1;
        uterm.push_back(key);
        return (int)uterm.size() - 1;
    }
    bool term_fits(const uint16_t *keys, int cnt) const {
        int fresh = 0;
        for (int i = 0; i < cnt; ++i) {
            bool found = false;
            for (uint16_t t : uterm) if (t == keys[i]) found = true;
            for (int j = 0; j < i; ++j) if (keys[j] == keys[i]) found = true;
            if (!found) ++fresh;
        }
        return (int)uterm.size() + fresh <= opt.ud_max;
    }
    static uint16_t tkey(uint8_t s1, uint8_t s2) {
        if (s2 != kNoSource && s2 < s1) std::swap(s1, s2);
        return (uint16_t)(s1 | (s2 << 8));
    }

    void emit_ud() {
        if (ud.empty()) return;
        HostOp &o = emit(OP_UDN);
        o.hdr.a = (uint8_t)uterm.size();
        uint64_t data = 0;
        for (size_t i = 0; i < uterm.size(); ++i) {
            if (i < 4) data |= (uint64_t)uterm[i] << (16 * i);
            else { o.hdr.sa = (uint8_t)(uterm[i] & 0xFF); o.hdr.sb = (uint8_t)(uterm[i] >> 8); }
        }
        o.hdr.data = data;
        o.pk = PK_UDN;
        o.ucon = ud;
        o.n_terms = (int)uterm.size();
        note_payload();
        f_used = true;
        ud.clear();
        uterm.clear();
    }

    // A 1-qubit diagonal (or the phases of Y) on a thread / tile-base bit.
    void add_ud1(const Src &s, int gate, uint8_t kind) {
        const uint16_t k1 = tkey(s.code, kNoSource);
        if (!term_fits(&k1, 1)) emit_ud();
        UContrib u;
        u.gate = gate;
        u.kind = kind;
        u.inv = s.inv != 0;
        u.t0 = (int8_t)term_slot(s.code, kNoSource);
        ud.push_back(u);
    }

    // A 2-qubit diagonal (CZ / CPHASE: one non-trivial entry) on two thread /
    // tile-base bits; only the terms its non-trivial entry needs are used.
    void add_ud2(const Src &s0, const Src &s1, int gate) {
        UContrib u;
        u.gate = gate;
        u.kind = UC_D2;
        for (int e = 0; e < 4; ++e) u.perm[e] = d4_index(e >> 1, e & 1, s0.inv, s1.inv);
        int es = 0;   // physical (x << 1) | y of the entry holding the gate's entry 3
        for (int e = 0; e < 4; ++e) if (u.perm[e] == 3) es = e;
        const bool need0 = es == 2 || es == 0, need1 = es == 1 || es == 0;
        uint16_t keys[3];
        int cnt = 0;
        if (need0) keys[cnt++] = tkey(s0.code, kNoSource);
        if (need1) keys[cnt++] = tkey(s1.code, kNoSource);
        keys[cnt++] = tkey(s0.code, s1.code);
        if (!term_fits(keys, cnt)) emit_ud();
        if (need0) u.t0 = (int8_t)term_slot(s0.code, kNoSource);
        if (need1) u.t1 = (int8_t)term_slot(s1.code, kNoSource);
        u.t01 = (int8_t)term_slot(s0.code, s1.code);
        ud.push_back(u);
    }

    // Register needs in this pass: a CNOT's control inside the tile is asked
    // for too, so that the CNOT becomes a compile-time register swap (a
    // control outside the tile is uniform per workgroup instead).
    uint64_t rneed_of(const CGate &g) const {
        uint64_t r = g.rneed;
        if (g.cls == G_CX && label_of[g.q0] >= 0) r |= bit(g.q0);
        return r;
    }

    bool absorbable(const CGate &g) const {
        const uint64_t rn = rneed_of(g);
        for (int qq = 0; qq < n; ++qq) {
            if (!((rn >> qq) & 1)) continue;
            const int l = label_of[qq];
            if (l < 0 || pos_reg[l] < 0) return false;
        }
        return true;
    }

    // Gate-local index of a 2-qubit diagonal entry from physical bits (x of
    // q0's position, y of q1's position) and the labels' XOR bits.
    static uint8_t d4_index(int x, int y, int inv0, int inv1) {
        return (uint8_t)(((x ^ inv0) << 1) | (y ^ inv1));
    }

    // Exchange register bits p and r (labels, pending products and the data).
    void rperm(int p, int r) {
        if (p == r) return;
        HostOp &o = emit(OP_RPERM);
        o.hdr.a = (uint8_t)p;
        o.hdr.b = (uint8_t)r;
        std::swap(reg_label[p], reg_label[r]);
        pos_reg[reg_label[p]] = p;
        pos_reg[reg_label[r]] = r;
        std::swap(pend[p], pend[r]);
        cur_layout = -1;
    }

    void apply(const CGate &g) {
        ++P.gates_applied;
        switch (g.cls) {
        case G_D1: {
            const Src s = src_of(g.q0);
            if (s.reg) {
                compose(s.p, Factor{FK_GATE, s.inv != 0, g.src}, PC_D, false);
            } else {
                add_ud1(s, g.src, UC_D1);
            }
            break;
        }
        case G_D2: {
            Src s0 = src_of(g.q0), s1 = src_of(g.q1);
            if (s0.reg) flush_nondiag(s0.p);   // may relabel: read the sources again
            if (s1.reg) flush_nondiag(s1.p);
            s0 = src_of(g.q0);
            s1 = src_of(g.q1);
            if (s0.reg && s1.reg) {
                // one non-trivial entry: a quarter of the slots
                int es = 0;
                for (int e = 0; e < 4; ++e)
                    if (d4_index(e >> 1, e & 1, s0.inv, s1.inv) == 3) es = e;
                HostOp &o = emit(OP_D2Q);
                o.hdr.a = (uint8_t)s0.p;
                o.hdr.b = (uint8_t)s1.p;
                o.hdr.sa = (uint8_t)(((es >> 1) & 1) | ((es & 1) << 1));
                o.pk = PK_G3;
                o.gate = g.src;
            } else if (s0.reg || s1.reg) {
                const Src &r = s0.reg ? s0 : s1;
                const Src &u = s0.reg ? s1 : s0;
                // e = (ub << 1) | rb; the gate's entry 3 sits at one e
                int es = 0;
                for (int e = 0; e < 4; ++e) {
                    const int ub = e >> 1, rb = e & 1;
                    const int gl = s0.reg ? d4_index(rb, ub, r.inv, u.inv) : d4_index(ub, rb, u.inv, r.inv);
                    if (gl == 3) es = e;
                }
                HostOp &o = emit(OP_D1HU);
                o.hdr.a = (uint8_t)r.p;
                o.hdr.b = (uint8_t)((es & 1) | (((es >> 1) & 1) << 1));
                o.hdr.sa = u.code;
                o.pk = PK_G3;
                o.gate = g.src;
            } else {
                add_ud2(s0, s1, g.src);
            }
            break;
        }
        case G_MARK: {
            for (int p = 0; p < opt.R; ++p) flush_nondiag(p);
            uint32_t lm = 0;     // the marked index's bits on the tile labels
            uint64_t pidx = 0;   // its bits off the tile, at their physical positions
            for (int l = 0; l < k; ++l)
                if ((g.index >> label_logi[l]) & 1) lm |= 1u << l;
            for (int qq = 0; qq < n; ++qq)
                if (label_of[qq] < 0 && ((g.index >> qq) & 1)) pidx |= bit(ph[qq]);
            const uint32_t phys = lm ^ xmask;
            int t = 0, j = 0;
            for (int s = 0; s < w; ++s) if ((phys >> thr_label[s]) & 1) t |= 1 << s;
            for (int p = 0; p < opt.R; ++p) if ((phys >> reg_label[p]) & 1) j |= 1 << p;
            HostOp &o = emit(OP_MARK);
            o.hdr.a = (uint8_t)j;
            o.hdr.sa = (uint8_t)(t & 0xFF);   // thread index: up to 2^10 threads
            o.hdr.sb = (uint8_t)(t >> 8);
            o.hdr.data = pidx ^ gxd;
            break;
        }
        case G_X: {
            const Src s = src_of(g.q0);
            if (label_of[g.q0] < 0) {
                gxd ^= bit(ph[g.q0]);   // off the tile: the global XOR, no data moves
                ++P.n_relabel;
            } else if (s.reg) {
                compose(s.p, Factor{FK_X, false, -1}, PC_A, true);
            } else {
                xmask ^= 1u << label_of[g.q0];
                cur_layout = -1;
                ++P.n_relabel;
            }
            break;
        }
        case G_Y: {
            const Src s = src_of(g.q0);
            if (s.reg) {
                compose(s.p, Factor{FK_GATE, s.inv != 0, g.src}, PC_A, false);
            } else {
                // Y = X diag(i, -i): the phases first, then the label flip
                // (off the tile: the global XOR bit)
                add_ud1(s, -1, UC_YDIAG);
                if (label_of[g.q0] < 0) {
                    gxd ^= bit(ph[g.q0]);
                } else {
                    xmask ^= 1u << label_of[g.q0];
                    cur_layout = -1;
                }
                ++P.n_relabel;
            }
            break;
        }
        case G_H: {
            const Src s = src_of(g.q0);
            compose(s.p, Factor{FK_H, s.inv != 0, -1}, s.inv ? PC_G : PC_H, false);
            break;
        }
        case G_DENSE1: {
            const Src s = src_of(g.q0);
            compose(s.p, Factor{FK_GATE, s.inv != 0, g.src}, PC_G, false);
            break;
        }
        case G_CX: {
            // flushing a pending pure X relabels (flips an XOR bit), so the
            // sources are read again after every flush
            const Src t = src_of(g.q1);
            flush(t.p);
            Src c = src_of(g.q0);
            if (c.reg) {
                flush_nondiag(c.p);
                c = src_of(g.q0);
                HostOp &o = emit(OP_CXR);
                o.hdr.a = (uint8_t)t.p;
                o.hdr.b = (uint8_t)c.p;
            } else if ((c.code & ~SRC_POS_MASK) == SRC_TILE) {
                HostOp &o = emit(OP_CXT);
                o.hdr.a = (uint8_t)t.p;
                o.hdr.sa = c.code;
            } else {
                HostOp &o = emit(OP_CXU);
                o.hdr.a = (uint8_t)t.p;
                o.hdr.sa = c.code;
            }
            // control acting on bit value 0 of the physical position:
            // CX_inverted = X_target * CX
            if (c.inv) compose(t.p, Factor{FK_X, false, -1}, PC_A, true);
            break;
        }
        case G_CCX: {
            // Toffoli as a monomial: swap the target's register pairs where
            // both controls hold 1. Register controls select slots; thread
            // and tile-base controls give a per-thread condition.
            flush(src_of(g.q2).p);
            for (int cq : {g.q0, g.q1}) {
                const Src c = src_of(cq);
                if (c.reg) flush_nondiag(c.p);
            }
            const Src t = src_of(g.q2);   // flushes may relabel: read again
            uint32_t cm = 0, cv = 0, uv = 0;
            uint8_t us[2] = {kNoSource, kNoSource};
            int nu = 0;
            for (int cq : {g.q0, g.q1}) {
                const Src c = src_of(cq);
                const uint32_t val = 1u ^ (uint32_t)c.inv;   // physical bit of logical 1
                if (c.reg) {
                    cm |= 1u << c.p;
                    cv |= val << c.p;
                } else {
                    us[nu] = c.code;
                    uv |= val << nu;
                    ++nu;
                }
            }
            HostOp &o = emit(OP_CCX);
            o.hdr.a = (uint8_t)t.p;
            o.hdr.b = (uint8_t)cm;
            o.hdr.sa = us[0];
            o.hdr.sb = us[1];
            o.hdr.data = cv | (uv << 8);
            break;
        }
        case G_DENSE2: {
            // a 4x4 on register bits 1 (q0) and 0 (q1)
            const int l0 = label_of[g.q0], l1 = label_of[g.q1];
            rperm(pos_reg[l0], 1);
            rperm(pos_reg[l1], 0);
            flush(0);
            flush(1);
            emit_ud();
            if (f_used) {
                emit(OP_APPLYF);
                f_used = false;
            }
            const int invm = (int)(((xmask >> l0) & 1) << 1 | ((xmask >> l1) & 1));
            const int per = opt.v ? 8 : 4;   // matrix entries per record payload
            HostOp &o = emit(OP_DENSE2);
            o.pk = PK_MAT4;
            o.gate = g.src;
            for (int e = 0; e < 4; ++e) o.perm[e] = (uint8_t)(e ^ invm);
            const uint8_t prm[4] = {o.perm[0], o.perm[1], o.perm[2], o.perm[3]};
            for (int e0 = per; e0 < 16; e0 += per) {
                HostOp &c = emit(OP_CONT);
                c.pk = PK_CONT;
                c.gate = g.src;
                c.hdr.a = (uint8_t)e0;
                std::memcpy(c.perm, prm, 4);
            }
            break;
        }
        case G_SWAP: {
            const int l0 = label_of[g.q0], l1 = label_of[g.q1];
            if (l0 < 0 || l1 < 0) {
                // a qubit off the tile: exchange the two qubits' places (the
                // tile label, or the physical bit off the tile) instead of
                // their data; the XOR bits stay with the places
                const int a = g.q0, b = g.q1;
                if (l0 >= 0) {          // a on label l0, b off the tile
                    const int pb = ph[b];
                    label_of[b] = l0; label_logi[l0] = b; label_of[a] = -1;
                    ph[a] = pb; lg[pb] = a; ph[b] = -1;
                } else if (l1 >= 0) {   // b on label l1, a off the tile
                    const int pa = ph[a];
                    label_of[a] = l1; label_logi[l1] = a; label_of[b] = -1;
                    ph[b] = pa; lg[pa] = b; ph[a] = -1;
                } else {
                    const int pa = ph[a], pb = ph[b];
                    ph[a] = pb; ph[b] = pa; lg[pa] = b; lg[pb] = a;
                }
                ++P.n_relabel;
                break;
            }
            const int r0 = pos_reg[l0], r1 = pos_reg[l1], t0 = pos_thr[l0], t1 = pos_thr[l1];
            if (r0 >= 0) reg_label[r0] = l1; else thr_label[t0] = l1;
            if (r1 >= 0) reg_label[r1] = l0; else thr_label[t1] = l0;
            pos_reg[l0] = r1; pos_thr[l0] = t1;
            pos_reg[l1] = r0; pos_thr[l1] = t0;
            const uint32_t b0 = (xmask >> l0) & 1, b1 = (xmask >> l1) & 1;
            if (b0 != b1) xmask ^= (1u << l0) | (1u << l1);
            cur_layout = -1;
            ++P.n_relabel;
            break;
        }
        default:
            --P.gates_applied;
            break;
        }
    }
};

}  // namespace

bool same_options(const PlanOptions &a, const PlanOptions &b) {
    return a.R == b.R && a.v == b.v && a.m == b.m && a.c == b.c && a.w_max == b.w_max &&
           a.fuse == b.fuse && a.remap == b.remap && a.max_dense == b.max_dense && a.auto_low == b.auto_low &&
           a.gen_h == b.gen_h && a.basis_known == b.basis_known &&
           (!a.basis_known || a.basis_j == b.basis_j) && a.gen_basis == b.gen_basis && a.ud_max == b.ud_max &&
           a.small_max == b.small_max && a.small_mode == b.small_mode;
}

Plan build_plan_auto(int n, const sv_gate *gates, size_t n_gates, const PlanOptions &opt) {
    Plan best = build_plan(n, gates, n_gates, opt);
    if (!opt.auto_low || best.small) return best;
    // Relative cost: a pass weighted by the streaming efficiency of its
    // contiguous runs (about 3% per halving of the run, measured), plus the
    // LDS exchanges (about 3% of a pass each, measured).
    auto cost = [](const Plan &p) {
        return (double)p.passes.size() * (1.0 + 0.03 * (6 - p.low)) + 0.03 * (double)p.n_exch;
    };
    PlanOptions o4 = opt;
    o4.c = 4;
    Plan alt = build_plan(n, gates, n_gates, o4);
    if (cost(alt) < cost(best)) best = std::move(alt);
    if (opt.v == 0) {
        // 16-byte amplitudes: 3 low qubits still give 128-byte runs, and the
        // extra free tile slot packs more gates into each pass
        PlanOptions o3 = opt;
        o3.c = 3;
        Plan alt3 = build_plan(n, gates, n_gates, o3);
        if (cost(alt3) < cost(best)) best = std::move(alt3);
    }
    return best;
}

Plan build_plan(int n, const sv_gate *gates, size_t n_gates, const PlanOptions &opt) {
    Plan P;
    P.n = n;
    P.low = opt.c;
    std::vector<CGate> cg;
    cg.reserve(n_gates);
    std::vector<int> kinds(n_gates);
    for (size_t i = 0; i < n_gates; ++i) kinds[i] = gates[i].kind;
    for (size_t i = 0; i < n_gates; ++i) {
        CGate c = classify(gates[i], n, (int)i);
        if (c.cls != G_NOP) cg.push_back(c);
    }

    int k = 0, w = 0;
    const bool tiled = tile_geometry(n, opt, k, w);
    const bool small = !tiled || (opt.small_mode == 2 && n <= opt.small_max);
    if (small) {
        P.small = true;
        for (const CGate &g : cg) {
            SmallOp so;
            std::memset(&so, 0, sizeof so);
            so.q0 = (uint8_t)(g.q0 < 0 ? 0 : g.q0);
            so.q1 = (uint8_t)(g.q1 < 0 ? 0 : g.q1);
            auto cblock = [&](ConstKind ck, int cnt) {
                ConstBlock b;
                b.kind = ck;
                b.gate = g.src;
                b.off = P.cstride;
                P.cblocks.push_back(b);
                P.cstride += (uint64_t)cnt;
                return b.off;
            };
            switch (g.cls) {
            case G_D1: so.code = SOP_D1; so.data = cblock(CK_D1, 4); break;
            case G_D2: so.code = SOP_D2; so.data = cblock(CK_D2, 8); break;
            case G_MARK: so.code = SOP_MARK; so.data = g.index; break;
            case G_X: so.code = SOP_X; break;
            case G_Y: so.code = SOP_Y; break;
            case G_CX: so.code = SOP_CX; break;
            case G_CCX: so.code = SOP_CCX; so.q2 = (uint8_t)g.q2; break;
            case G_SWAP: so.code = SOP_SWAP; break;
            case G_H: so.code = SOP_DENSE1; so.data = cblock(CK_HMAT, 8); break;
            case G_DENSE1: so.code = SOP_DENSE1; so.data = cblock(CK_DENSE1, 8); break;
            case G_DENSE2: so.code = SOP_DENSE2; so.data = cblock(CK_DENSE2, 32); break;
            default: continue;
            }
            P.sops.push_back(so);
            ++P.gates_applied;
        }
        return P;
    }

    // Leading Hadamards of a known basis state are generated, not applied.
    size_t start = 0;
    uint64_t gen_mask = 0;
    if (opt.gen_h && opt.basis_known) {
        while (start < cg.size() && cg[start].cls == G_H && !((gen_mask >> cg[start].q0) & 1)) {
            gen_mask |= bit(cg[start].q0);
            ++start;
        }
    }
    // Leading 1-qubit gates of a known basis state leave a product state. When
    // they are more than a run of Hadamards on distinct qubits, the first pass
    // generates amp[i] = prod_q u_q[bit q of i] instead (u_q: the qubit's
    // gates applied to its basis bit), the on-demand idea of the Hadamard
    // layer carried to any product state.
    bool product = false;
    auto qgates = std::make_shared<std::vector<std::vector<int>>>();
    if (opt.gen_h && opt.basis_known) {
        size_t s1 = 0;
        auto one_qubit = [](uint8_t c) { return c == G_D1 || c == G_H || c == G_DENSE1 || c == G_X || c == G_Y; };
        while (s1 < cg.size() && one_qubit(cg[s1].cls)) ++s1;
        if (s1 > start) {
            product = true;
            qgates->assign((size_t)n, {});
            for (size_t i = 0; i < s1; ++i) (*qgates)[(size_t)cg[i].q0].push_back(cg[i].src);
            P.n_gen_product = (int64_t)s1;
            start = s1;
            gen_mask = 0;
        }
    }
    // The first pass generates its input instead of reading it: a product
    // state, the Hadamard layer of a basis state, or the basis state itself
    // (empty mask: amp = [i == j]) when its memory was never written.
    const bool generate = opt.basis_known && ((opt.gen_h && gen_mask != 0) || opt.gen_basis || product);
    P.n_gen_h = popc(gen_mask);
    P.gates_applied += P.n_gen_h + P.n_gen_product;

    std::vector<int> order;
    for (size_t i = start; i < cg.size(); ++i) order.push_back((int)i);
    GateQueue pending;
    pending.order = &order;
    const int c = std::max(opt.v + 1, std::min(opt.c, k - 2));

    // Qubit remapping: logical qubit q lives at physical index bit phys[q].
    // Every tile contains the c lowest physical bits (contiguous HBM runs);
    // a pass may store its tile under any permutation of the tile's own
    // physical bits, so the store puts on the low bits the qubits the next
    // pass needs. Passes at the end put every qubit back (phys = identity).
    // A SWAP is a relabel (the two qubits exchange physical bits, no data
    // moves) wherever the pass's tile does not hold both of its qubits; that
    // needs the general qubit-to-bit map, which remapping maintains.
    std::vector<int> phys(n), logi(n);
    for (int q = 0; q < n; ++q) phys[q] = logi[q] = q;
    const bool remap = opt.remap && opt.fuse && n > k;
    if (remap)
        for (CGate &g : cg)
            if (g.cls == G_SWAP) g.qneed = 0;
    const uint64_t low_bits = bit(c) - 1;   // physical bits every tile holds
    auto identity = [&]() {
        for (int q = 0; q < n; ++q) if (phys[q] != q) return false;
        return true;
    };

    // Global XOR translation of addresses (physical bits): address a holds
    // the amplitude of index a ^ gx. X / Y on qubits off a pass's tile set
    // bits; a pass clears the bits of its tile (it stores them canonical).
    uint64_t gx = 0;
    // Spare tile slots (physical bits) take the bits set in gx.
    auto add_gx = [&](uint64_t Q) {
        for (int p = 0; p < n && popc(Q) < k; ++p)
            if ((gx >> p) & 1) Q |= bit(p);
        return Q;
    };
    // Spare tile slots take displaced qubits' home bits, following each
    // chain (the qubit at a home bit in the tile is displaced too: its own
    // home bit next), so that the store can put them home.
    auto add_homes = [&](uint64_t Q) {
        bool grew = true;
        while (grew && popc(Q) < k) {
            grew = false;
            for (int p = 0; p < n && popc(Q) < k; ++p) {
                if (!((Q >> p) & 1)) continue;
                const int x = logi[p];   // the qubit at p; its home bit is x
                if (x != p && !((Q >> x) & 1)) { Q |= bit(x); grew = true; }
            }
        }
        return Q;
    };

    // Tile set of a restoring pass: the low bits and the displacement chains
    // through them, then chains of the other displaced qubits, then bits of gx.
    auto restore_set = [&]() {
        uint64_t Q = add_homes(low_bits);
        for (int p = 0; p < n && popc(Q) < k; ++p) {
            if (logi[p] == p || ((Q >> p) & 1)) continue;
            Q = add_homes(Q | bit(p));
        }
        Q = add_gx(Q);
        for (int p = 0; p < n && popc(Q) < k; ++p) Q |= bit(p);
        return Q;
    };

    bool first = true;
    int restores = 0;
    while (true) {
        std::vector<int> taken;
        uint64_t Q;
        bool restoring = false;
        uint64_t want = 0;
        bool home_lanes = false;
        if (!pending.empty() || (first && generate)) {
            std::vector<int> ph_end = phys, lg_end = logi;   // the map after the pass's relabels
            Q = form_one_pass(cg, pending, n, k, opt, low_bits, true, taken, ph_end, lg_end);
            if (remap) {
                // qubits the next pass wants on the low bits: spare tile
                // slots take them so that the store can put them there
                if (!pending.empty()) {
                    std::vector<int> t2, ph2 = ph_end, lg2 = lg_end;
                    const uint64_t wp = form_one_pass(cg, pending, n, k, opt, 0, false, t2, ph2, lg2);
                    for (int p = 0; p < n; ++p)
                        if ((wp >> p) & 1) want |= bit(lg_end[p]);
                    for (int qq = 0; qq < n && popc(Q) < k; ++qq)
                        if ((want >> qq) & 1) Q |= bit(ph_end[qq]);
                } else {
                    home_lanes = true;   // last gate pass: head home
                }
            }
            if (pending.empty()) {
                // last gate pass: clear what it can of the XOR bits and the
                // displacements (chains through the end-of-pass map)
                Q = add_gx(Q);
                if (remap) {
                    std::vector<int> keep = logi;
                    logi = lg_end;
                    Q = add_homes(Q);
                    logi.swap(keep);
                }
            }
            for (int p = 0; p < n && popc(Q) < k; ++p) Q |= bit(p);
        } else if ((remap && !identity()) || gx != 0) {
            if (++restores > 2 * n) throw std::logic_error("qubit order not restored");
            Q = restore_set();
            restoring = true;
            home_lanes = true;
        } else {
            break;
        }

        PassCtx X(opt, P, cg, n, k, w);
        X.gkinds = kinds.data();
        X.ph = phys;
        X.lg = logi;
        for (int qq = 0; qq < 64; ++qq) X.label_of[qq] = -1;
        std::memset(X.q, 0, sizeof X.q);
        {
            int l = 0;
            for (int p = 0; p < n; ++p)   // labels in ascending physical order
                if ((Q >> p) & 1) {
                    X.q[l] = (uint8_t)p;
                    X.label_of[logi[p]] = l;
                    X.label_logi[l] = logi[p];
                    X.ph[logi[p]] = -1;   // on the tile: placed by its label
                    ++l;
                }
        }
        for (int l = 0; l < k; ++l) X.gpos[l] = X.q[l];

        DevPass dp;
        std::memset(&dp, 0, sizeof dp);
        dp.k = k;
        dp.w = w;
        dp.tiles = 1ull << (n - k);
        std::memcpy(dp.q, X.q, sizeof dp.q);
        dp.op_begin = (int)P.ops.size();
        dp.layout_begin = (int)P.layouts.size();
        X.layout_begin = dp.layout_begin;
        if (first && product) {
            // the product-state vectors head the pass's records (FP64 in
            // both precisions: the product of up to n factors is formed in
            // FP64 and rounded once)
            const int per = 2;   // qubits per record payload
            const int nrec = (n + per - 1) / per;
            for (int r = 0; r < nrec; ++r) {
                P.ops.emplace_back();
                HostOp &o = P.ops.back();
                o.hdr.code = r == 0 ? OP_GENP : OP_CONT;
                if (r == 0) {
                    o.hdr.a = (uint8_t)n;
                    o.hdr.b = (uint8_t)(nrec - 1);
                }
                o.pk = PK_PROD;
                o.qfirst = r * per;
                o.qcount = std::min(per, n - r * per);
                o.basis = opt.basis_j;
                o.qgates = qgates;
            }
        }
        X.op_floor = (int)P.ops.size();

        std::vector<int> rem = taken;
        const uint64_t U = X.U_labels();
        const int ru = opt.R - opt.v;
        auto labels_of = [&](uint64_t qmask) {
            uint64_t r = 0;
            for (int qq = 0; qq < n; ++qq)
                if (((qmask >> qq) & 1) && X.label_of[qq] >= 0) r |= bit(X.label_of[qq]);
            return r;
        };
        // a SWAP with a qubit off the tile relabels: the labels of later
        // gates on its qubits are known only once it is applied
        auto relabels = [&](const CGate &g) {
            return g.cls == G_SWAP && (X.label_of[g.q0] < 0 || X.label_of[g.q1] < 0);
        };

        // load layout: register labels from U, first-needed first
        uint64_t S0 = 0;
        {
            Blocker blk;
            for (int gi : rem) {
                const CGate &g = cg[gi];
                if (blk.conflicts(g) || relabels(g)) { blk.defer(g); continue; }
                const uint64_t nl = labels_of(X.rneed_of(g)) & U;
                if (popc(S0 | nl) <= ru) S0 |= nl;
                else blk.defer(g);
                if (popc(S0) == ru) break;
            }
            for (int lb = 0; lb < k && popc(S0) < ru; ++lb)
                if ((U >> lb) & 1) S0 |= bit(lb);
        }
        uint64_t tilemask = 0;   // the tile's physical bits
        for (int l = 0; l < k; ++l) tilemask |= bit(X.q[l]);
        X.gx_start = gx;
        X.gx_off = gx & ~tilemask;
        X.addr_xor = gx;          // the load reads the translated addresses
        X.load(X.storable(S0));
        X.layout_index();
        X.addr_xor = X.gx_off;    // later layouts: the tile's own bits canonical
        if (gx & tilemask) X.cur_layout = -1;

        while (!rem.empty()) {
            Blocker blk;
            std::vector<int> left;
            for (int gi : rem) {
                const CGate &g = cg[gi];
                if (!blk.conflicts(g) && X.absorbable(g)) {
                    X.apply(g);
                } else {
                    left.push_back(gi);
                    blk.defer(g);
                }
            }
            rem.swap(left);
            if (rem.empty()) break;
            // next register labels: needs of the next gates, in order
            const uint64_t regs = X.reg_labels();
            uint64_t S = 0;
            bool all_fit = true;
            Blocker b2;
            for (int gi : rem) {
                const CGate &g = cg[gi];
                if (b2.conflicts(g) || relabels(g)) { b2.defer(g); all_fit = false; continue; }
                const uint64_t nl = labels_of(X.rneed_of(g));
                if (popc(S | nl) <= opt.R) S |= nl;
                else { b2.defer(g); all_fit = false; }
            }
            X.flush_all();
            const uint64_t V = opt.v ? 1ull : 0ull;
            if (all_fit && (S & ~(U | V)) == 0 && popc(S | V) <= opt.R) {
                uint64_t su = S & U;
                for (int lb = 0; lb < k && popc(su) < ru; ++lb)   // keep current registers
                    if (((U & regs) >> lb) & 1) su |= bit(lb);
                for (int lb = 0; lb < k && popc(su) < ru; ++lb)
                    if ((U >> lb) & 1) su |= bit(lb);
                X.exchange_to(X.storable(su));
            } else {
                for (int lb = 0; lb < k && popc(S) < opt.R; ++lb)
                    if ((regs >> lb) & 1) S |= bit(lb);
                for (int lb = 0; lb < k && popc(S) < opt.R; ++lb) S |= bit(lb);
                X.exchange_to(X.general(S));
            }
        }
        X.flush_all();

        int sigma[32];   // new physical bit of every label
        for (int l = 0; l < k; ++l) sigma[l] = X.q[l];
        if (!remap) {
            if (!X.is_storable()) {
                uint64_t su = X.reg_labels() & U;
                while (popc(su) > ru) su &= su - 1;
                for (int lb = 0; lb < k && popc(su) < ru; ++lb)
                    if ((U >> lb) & 1) su |= bit(lb);
                X.exchange_to(X.storable(su));
            }
        } else {
            // The store may put the tile's qubits on any permutation of the
            // tile's physical bits. Qubits the next pass wants go to the low
            // bits (those already there stay); every other qubit goes home
            // when its home bit is in the tile; the rest keep their bits, or
            // take the bits left free. With `lanes_fixed` the labels on the
            // lane bits (the tile's lowest bits, which the store layout's
            // lanes address) keep them, so the store needs no exchange.
            uint64_t inP = tilemask;
            const bool free_exch = !X.is_storable();
            const uint64_t Wm = home_lanes ? 0 : want;
            const int nlane = opt.v + 6;
            auto build_sigma = [&](bool lanes_fixed, int *dst) {
                uint64_t used = 0;
                int made = 0;
                for (int l = 0; l < k; ++l) dst[l] = -1;
                auto put = [&](int l, int pos) { dst[l] = pos; used |= bit(pos); };
                if (lanes_fixed)
                    for (int l = 0; l < nlane && l < k; ++l) put(l, X.q[l]);
                if (!lanes_fixed) {
                    for (int l = 0; l < k; ++l)
                        if (((Wm >> X.label_logi[l]) & 1) && X.q[l] < c) put(l, X.q[l]);
                    for (int l = 0; l < k; ++l) {
                        if (dst[l] >= 0 || !((Wm >> X.label_logi[l]) & 1)) continue;
                        int a = 0;
                        while (a < c && ((used >> a) & 1)) ++a;
                        if (a == c) break;
                        put(l, a);
                        ++made;
                    }
                }
                for (int l = 0; l < k; ++l) {
                    const int x = X.label_logi[l];
                    if (dst[l] < 0 && ((inP >> x) & 1) && !((used >> x) & 1)) put(l, x);
                }
                for (int l = 0; l < k; ++l)
                    if (dst[l] < 0 && !((used >> X.q[l]) & 1)) put(l, X.q[l]);
                for (int l = 0; l < k; ++l) {
                    if (dst[l] >= 0) continue;
                    int pos = 0;
                    while (!((inP >> pos) & 1) || ((used >> pos) & 1)) ++pos;
                    put(l, pos);
                }
                return made;
            };
            const int made = build_sigma(false, sigma);
            bool lanes_move = false;
            for (int l = 0; l < nlane && l < k; ++l) lanes_move |= sigma[l] != X.q[l];
            // A lane change costs an exchange unless the pass ends with one.
            if (lanes_move && !home_lanes && !free_exch && made < 2) build_sigma(true, sigma);
            uint64_t hit = 0;
            for (int l = 0; l < k; ++l) hit |= bit(sigma[l]);
            if (hit != inP) throw std::logic_error("store permutation is not a bijection of the tile");
            int lane[6], reg0 = -1;
            for (int l = 0; l < k; ++l) {
                if (opt.v && sigma[l] == X.q[0]) reg0 = l;
                for (int s2 = 0; s2 < 6; ++s2)
                    if (sigma[l] == X.q[opt.v + s2]) lane[s2] = l;
            }
            X.settle_lanes(lane, reg0);
        }
        bool moved_any = false;
        for (int l = 0; l < k; ++l) moved_any |= X.gpos[l] != (uint8_t)sigma[l];
        if (moved_any) {   // the store addresses the labels at their new bits
            for (int l = 0; l < k; ++l) X.gpos[l] = (uint8_t)sigma[l];
            X.cur_layout = -1;
        }
        dp.store_layout = X.layout_index();
        // the map after the pass: qubits off the tile where the pass's
        // relabels left them, the tile's qubits at their labels' store bits
        for (int qq = 0; qq < n; ++qq)
            if (X.label_of[qq] < 0) {
                phys[qq] = X.ph[qq];
                logi[X.ph[qq]] = qq;
            }
        for (int l = 0; l < k; ++l) {
            phys[X.label_logi[l]] = sigma[l];
            logi[sigma[l]] = X.label_logi[l];
        }
        // stored in place: the tile's bits canonical, the others keep their
        // translation, flipped by the pass's X / Y off the tile
        gx = (gx ^ X.gxd) & ~tilemask;
        // In-place safety: without an exchange, nothing orders one wave's loads
        // before another wave's stores to the same tile.
        bool exch_in_pass = false;
        for (size_t oi = (size_t)dp.op_begin; oi < P.ops.size(); ++oi) {
            if (P.ops[oi].hdr.code == OP_EXCH) exch_in_pass = true;
            if (P.ops[oi].hdr.code == OP_DENSE2) dp.flags |= PASS_DENSE2;
        }
        if (!exch_in_pass && dp.store_layout != 0) dp.flags |= PASS_SYNC_STORE;

        if (first && product) {
            dp.flags |= PASS_GEN_PRODUCT;
            // the kernel reads the register bits' qubits from the load layout
            const DevLayout &L0 = P.layouts[(size_t)dp.layout_begin];
            for (int p = 0; p < opt.R; ++p)
                if (popc(L0.reg_goff[p]) != 1) throw std::logic_error("product generation: register bit without one global bit");
        } else if (first && generate) {
            dp.flags |= PASS_GENERATE;
            dp.gen_j = opt.basis_j;
            dp.gen_mask = gen_mask;
            dp.gen_scale = hadamard_magnitude(popc(gen_mask));
        }
        if (X.h_count > 0) {
            const double sc = hadamard_magnitude(X.h_count);
            if (X.first_payload >= 0) {
                P.ops[X.first_payload].scale *= sc;
            } else if (dp.flags & PASS_GENERATE) {
                dp.gen_scale *= sc;
            } else {
                HostOp &so = X.emit(OP_SCALE);
                so.pk = PK_SCALE;
                so.scale = sc;
            }
        }
        dp.op_end = (int)P.ops.size();
        dp.n_layouts = (int)P.layouts.size() - dp.layout_begin;
        P.passes.push_back(dp);
        if (restoring) ++P.n_restore;
        first = false;
    }
    return P;
}

// ---------------------------------------------------------------------------
// Gate constants (FP64, host libm), the product's own table.

static void gate_mat2(int kind, double t, cd m[4]) {
    const double r = 0.70710678118654752440;
    const cd I(0.0, 1.0);
    m[0] = 1.0; m[1] = 0.0; m[2] = 0.0; m[3] = 1.0;
    switch (kind) {
    case SV_GATE_X: m[0] = 0.0; m[1] = 1.0; m[2] = 1.0; m[3] = 0.0; break;
    case SV_GATE_Y: m[0] = 0.0; m[1] = -I; m[2] = I; m[3] = 0.0; break;
    case SV_GATE_Z: m[3] = -1.0; break;
    case SV_GATE_H: m[0] = r; m[1] = r; m[2] = r; m[3] = -r; break;
    case SV_GATE_S: m[3] = I; break;
    case SV_GATE_SDG: m[3] = -I; break;
    case SV_GATE_T: m[3] = cd(r, r); break;
    case SV_GATE_TDG: m[3] = cd(r, -r); break;
    case SV_GATE_RX: {
        const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
        m[0] = c; m[1] = cd(0.0, -s); m[2] = cd(0.0, -s); m[3] = c;
        break;
    }
    case SV_GATE_RY: {
        const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
        m[0] = c; m[1] = -s; m[2] = s; m[3] = c;
        break;
    }
    case SV_GATE_RZ: {
        const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
        m[0] = cd(c, -s); m[3] = cd(c, s);
        break;
    }
    case SV_GATE_P: m[3] = cd(std::cos(t), std::sin(t)); break;
    default: break;
    }
}

static void gate_diag4(int kind, double t, cd d[4]) {
    d[0] = d[1] = d[2] = d[3] = 1.0;
    if (kind == SV_GATE_CZ) d[3] = -1.0;
    else if (kind == SV_GATE_CPHASE) d[3] = cd(std::cos(t), std::sin(t));
}

static double gate_angle(const sv_gate &g, const double *params, size_t n_params, int b) {
    return g.param >= 0 ? params[(size_t)b * n_params + (size_t)g.param] : g.angle;
}

static void factor_mat(const Factor &f, const sv_gate *gates, const double *params,
                       size_t n_params, int b, cd m[4]) {
    const double r = 0.70710678118654752440;
    switch (f.kind) {
    case FK_GATE: {
        const sv_gate &g = gates[f.gate];
        if (g.kind == SV_GATE_U1) {
            const double *v = params + (size_t)b * n_params + (size_t)g.param;
            for (int e = 0; e < 4; ++e) m[e] = cd(v[2 * e], v[2 * e + 1]);
        } else {
            gate_mat2(g.kind, gate_angle(g, params, n_params, b), m);
        }
        break;
    }
    case FK_X: m[0] = 0.0; m[1] = 1.0; m[2] = 1.0; m[3] = 0.0; break;
    case FK_YDIAG: m[0] = cd(0.0, 1.0); m[1] = 0.0; m[2] = 0.0; m[3] = cd(0.0, -1.0); break;
    case FK_H: m[0] = r; m[1] = r; m[2] = r; m[3] = -r; break;
    }
    if (f.conj_x) {  // X M X: swap rows and columns
        std::swap(m[0], m[3]);
        std::swap(m[1], m[2]);
    }
}

template <typename R>
static void write_payload(DevOp &rec, const double *v, int count) {
    if ((size_t)count * sizeof(R) > sizeof rec.payload)
        throw std::logic_error("operation payload larger than its record");
    R *dst = reinterpret_cast<R *>(rec.payload);
    for (int i = 0; i < count; ++i) dst[i] = (R)v[i];
}

// FP32 rounding of unit-modulus constants (phases) with error diffusion.
// Rounding e^{i phi} to the nearest FP32 pair leaves a modulus error of a
// fixed sign for a given angle (fl32(cos pi/4)^2 + fl32(sin pi/4)^2 is
// 1 - 3.4e-8), so a circuit of many T gates would shrink the norm steadily.
// Among the pairs within one unit in the last place of the nearest one, take
// the one that brings the running sum of modulus errors closest to zero
// (ties: the closer pair). Other values round to nearest. The running sum
// starts at zero for every batch entry, so an entry's constants do not depend
// on the others.
struct PhaseRounder {
    double acc = 0.0;
    void pair(double re, double im, float &r, float &i) {
        const double m2 = re * re + im * im;
        r = (float)re;
        i = (float)im;
        if (std::fabs(m2 - 1.0) > 1e-12) return;
        float br = r, bi = i;
        double be = 0.0, bd = 0.0;
        bool have = false;
        for (int dr = -1; dr <= 1; ++dr) {
            for (int di = -1; di <= 1; ++di) {
                const float cr = dr ? std::nextafter(r, dr > 0 ? 2.0f : -2.0f) : r;
                const float ci = di ? std::nextafter(i, di > 0 ? 2.0f : -2.0f) : i;
                const double e = (double)cr * cr + (double)ci * ci - 1.0;
                const double d = std::fabs(cr - re) + std::fabs(ci - im);
                const double key = std::fabs(acc + e);
                if (!have || key < be || (key == be && d < bd)) {
                    br = cr; bi = ci; be = key; bd = d; have = true;
                }
            }
        }
        r = br;
        i = bi;
        acc += (double)r * r + (double)i * i - 1.0;
    }
    // `count` reals as (re, im) pairs
    void pairs(const double *v, int count, float *dst) {
        for (int k = 0; k + 1 < count; k += 2) pair(v[k], v[k + 1], dst[k], dst[k + 1]);
        if (count & 1) dst[count - 1] = (float)v[count - 1];
    }
};

void materialize_ops(const Plan &p, const sv_gate *gates, const double *params, size_t n_params,
                     int batch, bool f32, void *out) {
    DevOp *o = static_cast<DevOp *>(out);
    const size_t nops = p.ops.size();
    for (int b = 0; b < batch; ++b) {
        PhaseRounder ph;
        for (size_t i = 0; i < nops; ++i) {
            const HostOp &h = p.ops[i];
            DevOp rec = h.hdr;
            std::memset(rec.payload, 0, sizeof rec.payload);
            double v[16] = {0};   // up to 64 payload bytes of FP32 values
            int count = 0;
            switch (h.pk) {
            case PK_MAT2:
            case PK_MAT2RI:
            case PK_DIAG2: {
                cd M[4] = {1.0, 0.0, 0.0, 1.0};
                for (const Factor &f : h.factors) {
                    cd F[4];
                    factor_mat(f, gates, params, n_params, b, F);
                    const cd N[4] = {F[0] * M[0] + F[1] * M[2], F[0] * M[1] + F[1] * M[3],
                                     F[2] * M[0] + F[3] * M[2], F[2] * M[1] + F[3] * M[3]};
                    std::copy(N, N + 4, M);
                }
                if (h.pk == PK_MAT2) {
                    for (int e = 0; e < 4; ++e) { v[2 * e] = M[e].real() * h.scale; v[2 * e + 1] = M[e].imag() * h.scale; }
                    count = 8;
                } else if (h.pk == PK_MAT2RI) {
                    // R_rc = M_rc / i^(g_r + bt c): exact, the other part is zero
                    for (int e = 0; e < 4; ++e) {
                        const int r = e >> 1, col = e & 1;
                        const int ph = ((h.hdr.b >> r) & 1) + (col ? (h.hdr.b >> 2) & 1 : 0);
                        const double x = ph & 1 ? M[e].imag() : M[e].real();
                        v[e] = (ph & 2 ? -x : x) * h.scale;
                    }
                    count = 4;
                } else {
                    v[0] = M[0].real() * h.scale; v[1] = M[0].imag() * h.scale;
                    v[2] = M[3].real() * h.scale; v[3] = M[3].imag() * h.scale;
                    count = 4;
                }
                break;
            }
            case PK_D4: {
                const sv_gate &g = gates[h.gate];
                cd d[4];
                gate_diag4(g.kind, gate_angle(g, params, n_params, b), d);
                for (int e = 0; e < 4; ++e) {
                    v[2 * e] = d[h.perm[e]].real() * h.scale;
                    v[2 * e + 1] = d[h.perm[e]].imag() * h.scale;
                }
                count = 8;
                break;
            }
            case PK_SCALE: v[0] = h.scale; count = 1; break;
            case PK_PROD: {
                for (int t = 0; t < h.qcount; ++t) {
                    const int q = h.qfirst + t;
                    cd M[4] = {1.0, 0.0, 0.0, 1.0};
                    for (int gi : (*h.qgates)[(size_t)q]) {
                        cd F[4];
                        factor_mat(Factor{FK_GATE, false, gi}, gates, params, n_params, b, F);
                        const cd N[4] = {F[0] * M[0] + F[1] * M[2], F[0] * M[1] + F[1] * M[3],
                                         F[2] * M[0] + F[3] * M[2], F[2] * M[1] + F[3] * M[3]};
                        std::copy(N, N + 4, M);
                    }
                    const int bq = (int)((h.basis >> q) & 1);   // u = M e_bq: column bq
                    const cd u0 = M[bq], u1 = M[2 + bq];
                    v[4 * t] = u0.real(); v[4 * t + 1] = u0.imag();
                    v[4 * t + 2] = u1.real(); v[4 * t + 3] = u1.imag();
                }
                count = 4 * h.qcount;
                break;
            }
            case PK_MAT4:
            case PK_CONT: {
                // entries e0 .. e0 + per - 1 of the row-major 4x4, physical
                // (row, col) -> gate-local (perm[row], perm[col])
                const sv_gate &g = gates[h.gate];
                const double *mv = params + (size_t)b * n_params + (size_t)g.param;
                const int per = f32 ? 8 : 4;
                const int e0 = h.pk == PK_CONT ? h.hdr.a : 0;
                for (int t = 0; t < per; ++t) {
                    const int e = e0 + t, r = e >> 2, c = e & 3;
                    const int src = 4 * h.perm[r] + h.perm[c];
                    v[2 * t] = mv[2 * src];
                    v[2 * t + 1] = mv[2 * src + 1];
                }
                count = 2 * per;
                break;
            }
            case PK_SIDE: {
                cd M[4] = {1.0, 0.0, 0.0, 1.0};
                for (const Factor &f : h.factors) {
                    cd F[4];
                    factor_mat(f, gates, params, n_params, b, F);
                    const cd N[4] = {F[0] * M[0] + F[1] * M[2], F[0] * M[1] + F[1] * M[3],
                                     F[2] * M[0] + F[3] * M[2], F[2] * M[1] + F[3] * M[3]};
                    std::copy(N, N + 4, M);
                }
                const cd d = h.hdr.b ? M[3] : M[0];
                v[0] = d.real(); v[1] = d.imag();
                count = 2;
                break;
            }
            case PK_G3: {
                const sv_gate &g = gates[h.gate];
                cd d[4];
                gate_diag4(g.kind, gate_angle(g, params, n_params, b), d);
                v[0] = d[3].real(); v[1] = d[3].imag();
                count = 2;
                break;
            }
            case PK_UDN: {
                cd C = h.scale;
                cd r[kMaxUdTerms];
                for (int t = 0; t < kMaxUdTerms; ++t) r[t] = 1.0;
                for (const UContrib &u : h.ucon) {
                    cd P00, P01, P10, P11;
                    if (u.kind == UC_D2) {
                        const sv_gate &g = gates[u.gate];
                        cd d[4];
                        gate_diag4(g.kind, gate_angle(g, params, n_params, b), d);
                        P00 = d[u.perm[0]]; P01 = d[u.perm[1]]; P10 = d[u.perm[2]]; P11 = d[u.perm[3]];
                    } else {
                        cd m[4];
                        const Factor f{(uint8_t)(u.kind == UC_YDIAG ? FK_YDIAG : FK_GATE), u.inv, u.gate};
                        factor_mat(f, gates, params, n_params, b, m);
                        P00 = P01 = m[0];
                        P10 = P11 = m[3];
                    }
                    C *= P00;
                    if (u.t0 >= 0) r[u.t0] *= P10 / P00;
                    if (u.t1 >= 0) r[u.t1] *= P01 / P00;
                    if (u.t01 >= 0) r[u.t01] *= P11 * P00 / (P10 * P01);
                }
                v[0] = C.real(); v[1] = C.imag();
                for (int t = 0; t < h.n_terms; ++t) { v[2 + 2 * t] = r[t].real(); v[3 + 2 * t] = r[t].imag(); }
                count = 2 + 2 * h.n_terms;
                break;
            }
            default: break;
            }
            if (h.pk == PK_PROD) {
                write_payload<double>(rec, v, count);
            } else if (f32 && h.pk != PK_MAT2RI && h.pk != PK_SCALE) {
                // complex entries: phases through the error-diffusing rounding
                if ((size_t)count * sizeof(float) > sizeof rec.payload)
                    throw std::logic_error("operation payload larger than its record");
                ph.pairs(v, count, reinterpret_cast<float *>(rec.payload));
            } else if (f32) {
                write_payload<float>(rec, v, count);
            } else {
                write_payload<double>(rec, v, count);
            }
            o[(size_t)b * nops + i] = rec;
        }
    }
}

void materialize_consts(const Plan &p, const sv_gate *gates, const double *params,
                        size_t n_params, int batch, bool f32, void *out) {
    std::vector<double> row(p.cstride);
    for (int b = 0; b < batch; ++b) {
        std::fill(row.begin(), row.end(), 0.0);
        for (const ConstBlock &cb : p.cblocks) {
            double *d = row.data() + cb.off;
            const sv_gate &g = gates[cb.gate];
            const double t = gate_angle(g, params, n_params, b);
            if (cb.kind == CK_D2) {
                cd e[4];
                gate_diag4(g.kind, t, e);
                for (int i = 0; i < 4; ++i) { d[2 * i] = e[i].real(); d[2 * i + 1] = e[i].imag(); }
            } else if (cb.kind == CK_DENSE2 || (cb.kind == CK_DENSE1 && g.kind == SV_GATE_U1)) {
                const double *mv = params + (size_t)b * n_params + (size_t)g.param;
                std::memcpy(d, mv, (cb.kind == CK_DENSE2 ? 32 : 8) * sizeof(double));
            } else {
                cd m[4];
                gate_mat2(cb.kind == CK_HMAT ? (int)SV_GATE_H : g.kind, t, m);
                if (cb.kind == CK_D1) {
                    d[0] = m[0].real(); d[1] = m[0].imag(); d[2] = m[3].real(); d[3] = m[3].imag();
                } else {
                    for (int i = 0; i < 4; ++i) { d[2 * i] = m[i].real(); d[2 * i + 1] = m[i].imag(); }
                }
            }
        }
        if (f32) {
            // every constant block holds (re, im) pairs
            float *o = static_cast<float *>(out) + (size_t)b * p.cstride;
            PhaseRounder ph;
            ph.pairs(row.data(), (int)p.cstride, o);
        } else {
            double *o = static_cast<double *>(out) + (size_t)b * p.cstride;
            if (p.cstride) std::memcpy(o, row.data(), p.cstride * sizeof(double));
        }
    }
}

}  // namespace sv
