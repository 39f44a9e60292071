// Gate classification, pass planning and constant tables (host side).
//
// Classification follows the paper's observation (Sec. II-C, Table 1) that
// most gates are sparse: diagonal and monomial gates are applied from their
// gate-local non-zeros only (DAX: value + index, Sec. III-A1), Hadamards from
// one magnitude plus index-derived signs (RH, Sec. III-B1), and only the rest
// as dense 2x2 / 4x4 butterflies. Where the paper composes a stage's gates into
// one compressed operator before a single matrix-vector product (Sec. III-A2),
// the planner composes a run of gates into one pass over HBM instead: the
// operator is never formed, only the schedule.
#include "sv_planner.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "sv_swizzle.hpp"

namespace sv {

static inline int popc(uint64_t x) { return __builtin_popcountll(x); }
static inline uint64_t bit(int q) { return 1ull << q; }

static bool is_angled(int kind) {
    return kind == SV_GATE_RX || kind == SV_GATE_RY || kind == SV_GATE_RZ ||
           kind == SV_GATE_P || kind == SV_GATE_CPHASE;
}
static bool is_2q(int kind) {
    return kind == SV_GATE_CNOT || kind == SV_GATE_CZ || kind == SV_GATE_SWAP ||
           kind == SV_GATE_CPHASE;
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
        if (g.param >= 0) {
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
    case SV_GATE_RX: case SV_GATE_RY: c.cls = G_DENSE1; break;
    case SV_GATE_CNOT: c.cls = G_CX; break;
    case SV_GATE_CZ: case SV_GATE_CPHASE: c.cls = G_D2; break;
    case SV_GATE_SWAP: c.cls = G_SWAP; break;
    case SV_GATE_MARK: c.cls = G_MARK; c.index = g.index; break;
    default: c.cls = G_NOP; break;
    }
    switch (c.cls) {
    case G_D1: c.diag = true; c.support = bit(c.q0); break;
    case G_D2: c.diag = true; c.support = bit(c.q0) | bit(c.q1); break;
    case G_MARK: c.diag = true; c.support = (n >= 64) ? ~0ull : (bit(n) - 1); break;
    case G_X: case G_Y: case G_H: case G_DENSE1:
        c.support = bit(c.q0); c.need = bit(c.q0); break;
    case G_CX: c.support = bit(c.q0) | bit(c.q1); c.need = bit(c.q1); break;
    case G_SWAP: case G_DENSE2:
        c.support = bit(c.q0) | bit(c.q1); c.need = c.support; break;
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

static bool is_dense(GClass c) { return c == G_DENSE1 || c == G_DENSE2; }

namespace {

struct PassCtx {
    const PlanOptions &opt;
    Plan &P;
    const std::vector<CGate> &cg;
    int n, k, w;
    uint8_t q[32];
    int local_of[64];
    int pass_layout_begin = 0;
    DevLayout cur;
    int reg_of_local[32];   // register bit of a tile-local bit, -1 if a thread bit
    int thr_of_local[32];

    PassCtx(const PlanOptions &o, Plan &p, const std::vector<CGate> &g, int n_, int k_, int w_)
        : opt(o), P(p), cg(g), n(n_), k(k_), w(w_) {}

    uint64_t U_mask() const {  // local bits that may hold registers in a storable layout
        uint64_t u = 0;
        for (int l = opt.v + 6; l < k; ++l) u |= bit(l);
        return u;
    }
    uint64_t V_mask() const { return opt.v ? 1ull : 0ull; }
    uint64_t lanes_mask() const {
        uint64_t u = 0;
        for (int l = opt.v; l < opt.v + 6; ++l) u |= bit(l);
        return u;
    }
    uint64_t to_local(uint64_t qmask) const {
        uint64_t r = 0;
        for (int qq = 0; qq < n; ++qq)
            if ((qmask >> qq) & 1) r |= bit(local_of[qq]);
        return r;
    }

    // regs_u: R - v tile-local bits from U_mask().
    DevLayout storable(uint64_t regs_u) const {
        DevLayout L;
        std::memset(&L, 0, sizeof L);
        int p = 0;
        for (int l = 0; l < opt.v; ++l) L.reg_local[p++] = (uint8_t)l;
        for (int l = 0; l < k; ++l)
            if ((regs_u >> l) & 1) L.reg_local[p++] = (uint8_t)l;
        int s = 0;
        for (int l = opt.v; l < opt.v + 6; ++l) L.thr_local[s++] = (uint8_t)l;
        const uint64_t rest = U_mask() & ~regs_u;
        for (int l = 0; l < k; ++l)
            if ((rest >> l) & 1) L.thr_local[s++] = (uint8_t)l;
        return L;
    }

    // regs: R tile-local bits; lanes 0..m-1 get thread bits whose swizzle
    // images are linearly independent (conflict-free LDS rows).
    DevLayout general(uint64_t regs) const {
        DevLayout L;
        std::memset(&L, 0, sizeof L);
        int p = 0;
        for (int l = 0; l < k; ++l)      // ascending: local bit 0 lands on register 0
            if ((regs >> l) & 1) L.reg_local[p++] = (uint8_t)l;
        std::vector<int> thr;
        for (int l = 0; l < k; ++l)
            if (!((regs >> l) & 1)) thr.push_back(l);
        std::vector<int> lanes;
        uint32_t basis[8] = {0};  // GF(2) basis indexed by leading bit
        std::vector<int> others;
        for (int l : thr) {
            uint32_t x = swz_image(l, opt.m);
            for (int b = opt.m - 1; b >= 0 && x; --b) {
                if (!((x >> b) & 1)) continue;
                if (basis[b]) x ^= basis[b];
                else { basis[b] = x; break; }
            }
            if (x && (int)lanes.size() < opt.m) lanes.push_back(l);
            else others.push_back(l);
        }
        int s = 0;
        for (int l : lanes) L.thr_local[s++] = (uint8_t)l;
        for (int l : others) L.thr_local[s++] = (uint8_t)l;
        return L;
    }

    bool is_storable(const DevLayout &L) const {
        for (int p = 0; p < opt.v; ++p)
            if (L.reg_local[p] != p) return false;
        for (int s = 0; s < 6; ++s)
            if (L.thr_local[s] != opt.v + s) return false;
        return true;
    }

    uint64_t reg_mask(const DevLayout &L) const {
        uint64_t r = 0;
        for (int p = 0; p < opt.R; ++p) r |= bit(L.reg_local[p]);
        return r;
    }

    void set_current(const DevLayout &L) {
        cur = L;
        for (int l = 0; l < 32; ++l) reg_of_local[l] = thr_of_local[l] = -1;
        for (int p = 0; p < opt.R; ++p) reg_of_local[L.reg_local[p]] = p;
        for (int s = 0; s < w; ++s) thr_of_local[L.thr_local[s]] = s;
    }

    int add_layout(const DevLayout &L) {
        P.layouts.push_back(L);
        return (int)P.layouts.size() - 1 - pass_layout_begin;
    }

    uint8_t src_of(int qubit) const {
        const int l = local_of[qubit];
        if (l >= 0) {
            if (reg_of_local[l] >= 0) return (uint8_t)(SRC_REG | reg_of_local[l]);
            return (uint8_t)(SRC_THR | thr_of_local[l]);
        }
        return (uint8_t)(SRC_TILE | qubit);
    }
    int reg_of(int qubit) const { return reg_of_local[local_of[qubit]]; }

    uint64_t add_const(ConstKind kind, int gate, int count, bool swap_bits = false,
                       double scale = 1.0) {
        ConstBlock b;
        b.kind = kind;
        b.gate = gate;
        b.scale = scale;
        b.off = P.cstride;
        b.swap_bits = swap_bits;
        P.cblocks.push_back(b);
        P.cstride += (uint64_t)count;
        return b.off;
    }

    // Emit the op of gate g in the current layout. Returns the index of its
    // constant block in P.cblocks, or -1.
    int emit(const CGate &g, int &h_count) {
        DevOp op;
        std::memset(&op, 0, sizeof op);
        int cb = -1;
        switch (g.cls) {
        case G_D1:
            op.code = OP_D1;
            op.sa = src_of(g.q0);
            cb = (int)P.cblocks.size();
            op.data = add_const(CK_D1, g.src, 4);
            break;
        case G_D2:
            op.code = OP_D2;
            op.sa = src_of(g.q0);
            op.sb = src_of(g.q1);
            cb = (int)P.cblocks.size();
            op.data = add_const(CK_D2, g.src, 8);
            break;
        case G_MARK: {
            op.code = OP_MARK;
            uint64_t qmask = 0;
            for (int l = 0; l < k; ++l) qmask |= bit(q[l]);
            op.data = g.index & ~qmask;
            int t = 0, j = 0;
            for (int l = 0; l < k; ++l) {
                if (!((g.index >> q[l]) & 1)) continue;
                if (reg_of_local[l] >= 0) j |= 1 << reg_of_local[l];
                else t |= 1 << thr_of_local[l];
            }
            op.a = (uint8_t)j;
            op.b = (uint8_t)t;
            break;
        }
        case G_X: op.code = OP_X; op.a = (uint8_t)reg_of(g.q0); break;
        case G_Y: op.code = OP_Y; op.a = (uint8_t)reg_of(g.q0); break;
        case G_H: op.code = OP_H; op.a = (uint8_t)reg_of(g.q0); ++h_count; break;
        case G_DENSE1:
            op.code = OP_DENSE1;
            op.a = (uint8_t)reg_of(g.q0);
            cb = (int)P.cblocks.size();
            op.data = add_const(CK_DENSE1, g.src, 8);
            break;
        case G_CX:
            op.code = OP_CX;
            op.a = (uint8_t)reg_of(g.q1);
            op.sa = src_of(g.q0);
            break;
        case G_SWAP: {
            int a = reg_of(g.q0), b = reg_of(g.q1);
            if (a < b) std::swap(a, b);
            op.code = OP_SWAP;
            op.a = (uint8_t)a;
            op.b = (uint8_t)b;
            break;
        }
        case G_DENSE2: {
            int a = reg_of(g.q0), b = reg_of(g.q1);
            const bool sw = a < b;
            if (sw) std::swap(a, b);
            op.code = OP_DENSE2;
            op.a = (uint8_t)a;
            op.b = (uint8_t)b;
            cb = (int)P.cblocks.size();
            op.data = add_const(CK_DENSE2, g.src, 32, sw);
            break;
        }
        default:
            return -1;
        }
        P.ops.push_back(op);
        ++P.gates_applied;
        return cb;
    }
};

}  // namespace

// Split `gates` into passes; each entry lists indices into cg.
static std::vector<std::vector<int>> form_passes(const std::vector<CGate> &cg,
                                                 const std::vector<int> &order, int n, int k,
                                                 const PlanOptions &opt, int c,
                                                 std::vector<uint64_t> &qsets) {
    std::vector<std::vector<int>> passes;
    std::vector<int> pending = order;
    const uint64_t all = (n >= 64) ? ~0ull : (bit(n) - 1);
    const uint64_t low = (c >= 64) ? ~0ull : (bit(c) - 1);
    while (!pending.empty()) {
        uint64_t Q = low & all;
        Blocker blk;
        std::vector<int> taken, deferred;
        int dense = 0;
        bool closed = false;
        for (size_t i = 0; i < pending.size(); ++i) {
            const int gi = pending[i];
            const CGate &g = cg[gi];
            if (closed) { deferred.push_back(gi); continue; }
            bool take = false;
            if (!blk.conflicts(g)) {
                const uint64_t need = g.need;
                const bool dense_ok = !is_dense(g.cls) || dense < opt.max_dense;
                if (dense_ok && (need & ~Q) == 0) take = true;
                else if (dense_ok && popc(Q | need) <= k) { Q |= need; take = true; }
            }
            if (take) {
                taken.push_back(gi);
                if (is_dense(g.cls)) ++dense;
                if (!opt.fuse) closed = true;
            } else {
                deferred.push_back(gi);
                blk.defer(g);
                if ((blk.nondiag & all) == all) closed = true;  // nothing can move past
            }
        }
        // fill Q up to k qubits with the lowest ones not yet in it
        for (int qq = 0; qq < n && popc(Q) < k; ++qq) Q |= bit(qq);
        passes.push_back(taken);
        qsets.push_back(Q);
        pending.swap(deferred);
    }
    return passes;
}

static double hadamard_magnitude(int h) {
    // 2^(-h/2): exact for even h, one rounding of 1/sqrt(2) for odd h
    double s = std::ldexp(1.0, -(h / 2));
    if (h & 1) s *= 0.70710678118654752440;
    return s;
}

Plan build_plan(int n, const sv_gate *gates, size_t n_gates, const PlanOptions &opt) {
    Plan P;
    P.n = n;
    std::vector<CGate> cg;
    cg.reserve(n_gates);
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
                b.scale = 1.0;
                b.off = P.cstride;
                b.swap_bits = false;
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
    const bool generate = opt.basis_known && opt.gen_h && gen_mask != 0;
    P.n_gen_h = popc(gen_mask);
    P.gates_applied += P.n_gen_h;

    std::vector<int> order;
    for (size_t i = start; i < cg.size(); ++i) order.push_back((int)i);
    const int c = std::max(opt.v + 1, std::min(opt.c, k - 2));
    std::vector<uint64_t> qsets;
    std::vector<std::vector<int>> groups = form_passes(cg, order, n, k, opt, c, qsets);
    if (groups.empty() && generate) {
        groups.emplace_back();
        uint64_t Q = 0;
        for (int qq = 0; qq < k; ++qq) Q |= bit(qq);
        qsets.push_back(Q);
    }

    for (size_t pi = 0; pi < groups.size(); ++pi) {
        PassCtx X(opt, P, cg, n, k, w);
        const uint64_t Q = qsets[pi];
        int l = 0;
        for (int qq = 0; qq < 64; ++qq) X.local_of[qq] = -1;
        std::memset(X.q, 0, sizeof X.q);
        for (int qq = 0; qq < n; ++qq)
            if ((Q >> qq) & 1) { X.q[l] = (uint8_t)qq; X.local_of[qq] = l; ++l; }

        DevPass dp;
        std::memset(&dp, 0, sizeof dp);
        dp.k = k;
        dp.w = w;
        dp.tiles = 1ull << (n - k);
        std::memcpy(dp.q, X.q, sizeof dp.q);
        dp.op_begin = (int)P.ops.size();
        dp.layout_begin = (int)P.layouts.size();
        X.pass_layout_begin = dp.layout_begin;

        std::vector<int> rem = groups[pi];
        const uint64_t U = X.U_mask();
        const int ru = opt.R - opt.v;

        // initial (load) layout: register bits from U, first-needed first
        uint64_t S0 = 0;
        {
            Blocker blk;
            for (int gi : rem) {
                const CGate &g = cg[gi];
                if (blk.conflicts(g)) { blk.defer(g); continue; }
                const uint64_t nl = X.to_local(g.need) & U;
                if (popc(S0 | nl) <= ru) S0 |= nl;
                else blk.defer(g);
                if (popc(S0) == ru) break;
            }
            for (int lb = 0; lb < k && popc(S0) < ru; ++lb)
                if ((U >> lb) & 1) S0 |= bit(lb);
        }
        DevLayout L0 = X.storable(S0);
        X.add_layout(L0);
        X.set_current(L0);

        int h_count = 0;
        int first_cb = -1;
        while (true) {
            // absorb every gate that can run in the current layout
            const uint64_t regs = X.reg_mask(X.cur);
            Blocker blk;
            std::vector<int> left;
            for (int gi : rem) {
                const CGate &g = cg[gi];
                if (!blk.conflicts(g) && (X.to_local(g.need) & ~regs) == 0) {
                    const int cb = X.emit(g, h_count);
                    if (cb >= 0 && first_cb < 0) first_cb = cb;
                } else {
                    left.push_back(gi);
                    blk.defer(g);
                }
            }
            rem.swap(left);
            if (rem.empty()) break;
            // next register set: needs of the next gates, in order
            uint64_t S = 0;
            bool all_fit = true;
            Blocker b2;
            for (int gi : rem) {
                const CGate &g = cg[gi];
                if (b2.conflicts(g)) { b2.defer(g); all_fit = false; continue; }
                const uint64_t nl = X.to_local(g.need);
                if (popc(S | nl) <= opt.R) S |= nl;
                else { b2.defer(g); all_fit = false; }
            }
            DevLayout NL;
            const uint64_t V = X.V_mask();
            if (all_fit && (S & ~(U | V)) == 0 && popc(S | V) <= opt.R) {
                uint64_t su = S & U;
                for (int lb = 0; lb < k && popc(su) < ru; ++lb)   // keep current registers
                    if (((U & regs) >> lb) & 1) su |= bit(lb);
                for (int lb = 0; lb < k && popc(su) < ru; ++lb)
                    if ((U >> lb) & 1) su |= bit(lb);
                NL = X.storable(su);
            } else {
                for (int lb = 0; lb < k && popc(S) < opt.R; ++lb)
                    if ((regs >> lb) & 1) S |= bit(lb);
                for (int lb = 0; lb < k && popc(S) < opt.R; ++lb) S |= bit(lb);
                NL = X.general(S);
            }
            DevOp ex;
            std::memset(&ex, 0, sizeof ex);
            ex.code = OP_EXCH;
            ex.a = (uint8_t)X.add_layout(NL);
            P.ops.push_back(ex);
            ++P.n_exch;
            X.set_current(NL);
        }
        if (!X.is_storable(X.cur)) {
            uint64_t su = X.reg_mask(X.cur) & U;
            for (int lb = 0; lb < k && popc(su) < ru; ++lb)
                if ((U >> lb) & 1) su |= bit(lb);
            while (popc(su) > ru) su &= su - 1;
            DevLayout NL = X.storable(su);
            DevOp ex;
            std::memset(&ex, 0, sizeof ex);
            ex.code = OP_EXCH;
            ex.a = (uint8_t)X.add_layout(NL);
            P.ops.push_back(ex);
            ++P.n_exch;
            X.set_current(NL);
        }

        if (pi == 0 && generate) {
            dp.flags |= PASS_GENERATE;
            dp.gen_j = opt.basis_j;
            dp.gen_mask = gen_mask;
            dp.gen_scale = hadamard_magnitude(popc(gen_mask));
        }
        if (h_count > 0) {
            const double s = hadamard_magnitude(h_count);
            if (first_cb >= 0) {
                P.cblocks[first_cb].scale *= s;
            } else if (dp.flags & PASS_GENERATE) {
                dp.gen_scale *= s;
            } else {
                DevOp so;
                std::memset(&so, 0, sizeof so);
                so.code = OP_SCALE;
                so.data = X.add_const(CK_SCALE, -1, 1, false, s);
                P.ops.push_back(so);
            }
        }
        dp.op_end = (int)P.ops.size();
        P.passes.push_back(dp);
    }
    return P;
}

// ---------------------------------------------------------------------------
// Gate constants (FP64, host libm), the product's own table.

static void gate_d1(int kind, double t, double *d) {
    const double r = 0.70710678118654752440;
    double v[4] = {1, 0, 1, 0};
    switch (kind) {
    case SV_GATE_Z: v[2] = -1; break;
    case SV_GATE_S: v[2] = 0; v[3] = 1; break;
    case SV_GATE_SDG: v[2] = 0; v[3] = -1; break;
    case SV_GATE_T: v[2] = r; v[3] = r; break;
    case SV_GATE_TDG: v[2] = r; v[3] = -r; break;
    case SV_GATE_RZ: {
        const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
        v[0] = c; v[1] = -s; v[2] = c; v[3] = s;
        break;
    }
    case SV_GATE_P: v[2] = std::cos(t); v[3] = std::sin(t); break;
    default: break;
    }
    std::memcpy(d, v, sizeof v);
}

static void gate_d2(int kind, double t, double *d) {
    double v[8] = {1, 0, 1, 0, 1, 0, 1, 0};
    if (kind == SV_GATE_CZ) v[6] = -1;
    else if (kind == SV_GATE_CPHASE) { v[6] = std::cos(t); v[7] = std::sin(t); }
    std::memcpy(d, v, sizeof v);
}

static void gate_dense1(int kind, double t, double *m) {
    const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
    double v[8] = {0};
    if (kind == SV_GATE_RX) {         // [[c, -is], [-is, c]]
        v[0] = c; v[3] = -s; v[5] = -s; v[6] = c;
    } else if (kind == SV_GATE_RY) {  // [[c, -s], [s, c]]
        v[0] = c; v[2] = -s; v[4] = s; v[6] = c;
    } else if (kind == SV_GATE_H) {
        const double r = 0.70710678118654752440;
        v[0] = r; v[2] = r; v[4] = r; v[6] = -r;
    }
    std::memcpy(m, v, sizeof v);
}

void materialize_consts(const Plan &p, const sv_gate *gates, const double *params,
                        size_t n_params, int batch, bool f32, void *out) {
    std::vector<double> row(p.cstride);
    for (int b = 0; b < batch; ++b) {
        std::fill(row.begin(), row.end(), 0.0);
        for (const ConstBlock &cb : p.cblocks) {
            double *d = row.data() + cb.off;
            double t = 0.0;
            int kind = -1;
            if (cb.gate >= 0) {
                const sv_gate &g = gates[cb.gate];
                kind = g.kind;
                t = g.param >= 0 ? params[(size_t)b * n_params + (size_t)g.param] : g.angle;
            }
            int cnt = 0;
            switch (cb.kind) {
            case CK_D1: gate_d1(kind, t, d); cnt = 4; break;
            case CK_D2: gate_d2(kind, t, d); cnt = 8; break;
            case CK_DENSE1: gate_dense1(kind, t, d); cnt = 8; break;
            case CK_HMAT: gate_dense1(SV_GATE_H, 0.0, d); cnt = 8; break;
            case CK_SCALE: d[0] = 1.0; cnt = 1; break;
            case CK_DENSE2: cnt = 32; break;  // no 4x4 dense kind in this gate set yet
            }
            if (cb.kind == CK_D2 && cb.swap_bits) std::swap_ranges(d + 2, d + 4, d + 4);
            for (int i = 0; i < cnt; ++i) d[i] *= cb.scale;
        }
        if (f32) {
            float *o = static_cast<float *>(out) + (size_t)b * p.cstride;
            for (uint64_t i = 0; i < p.cstride; ++i) o[i] = (float)row[i];
        } else {
            double *o = static_cast<double *>(out) + (size_t)b * p.cstride;
            std::memcpy(o, row.data(), p.cstride * sizeof(double));
        }
    }
}

}  // namespace sv
