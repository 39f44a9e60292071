// Host lowering of composite Table 1 gates (see sv_lower.hpp for the rules).
#include "sv_lower.hpp"

#include <cmath>

namespace sv {

namespace {

const double kPi = 3.14159265358979323846;

sv_gate mk(int kind, int q0, int q1 = -1, double angle = 0.0, int param = -1, uint64_t index = 0) {
    sv_gate g;
    g.kind = kind;
    g.q0 = q0;
    g.q1 = q1;
    g.param = param;
    g.angle = angle;
    g.index = index;
    return g;
}

// An angle: a fixed value, or `scale` times parameter column `src`.
struct Ang {
    int src = -1;
    double scale = 1.0;
    double value = 0.0;
    Ang times(double k) const { return Ang{src, scale * k, value * k}; }
};
Ang fixed(double v) { return Ang{-1, 1.0, v}; }

struct Lowerer {
    size_t n_params;
    Lowering &L;

    void put(int kind, int q0, int q1 = -1, uint64_t index = 0) { L.gates.push_back(mk(kind, q0, q1, 0.0, -1, index)); }
    void put(int kind, int q0, int q1, Ang a) {
        if (a.src < 0) {
            L.gates.push_back(mk(kind, q0, q1, a.value));
        } else if (a.scale == 1.0) {
            L.gates.push_back(mk(kind, q0, q1, 0.0, a.src));
        } else {
            const int col = (int)(n_params + L.src.size());
            L.src.push_back(a.src);
            L.scale.push_back(a.scale);
            L.gates.push_back(mk(kind, q0, q1, 0.0, col));
        }
    }
    // angle j of gate g: its own angle or parameter (j = 0), or column param + j
    static Ang angle(const sv_gate &g, int j = 0) {
        if (g.param < 0) return fixed(g.angle);
        return Ang{g.param + j, 1.0, 0.0};
    }

    // RZZ(x) = CPHASE(-2x) P_b(x) RZ_a(x)
    void rzz(int a, int b, Ang x) {
        put(SV_GATE_RZ, a, -1, x);
        put(SV_GATE_P, b, -1, x);
        put(SV_GATE_CPHASE, a, b, x.times(-2.0));
    }
    // RXX(x) = (H (x) H) RZZ(x) (H (x) H)
    void rxx(int a, int b, Ang x) {
        put(SV_GATE_H, a);
        put(SV_GATE_H, b);
        rzz(a, b, x);
        put(SV_GATE_H, a);
        put(SV_GATE_H, b);
    }
    // RZX(x) = (I (x) H) RZZ(x) (I (x) H): Z on a, X on b
    void rzx(int a, int b, Ang x) {
        put(SV_GATE_H, b);
        rzz(a, b, x);
        put(SV_GATE_H, b);
    }
    // controlled U(t, p, l) = CPHASE(p) CRY(t) CPHASE(l), with
    // CRY(t) = CNOT RY_t(-t/2) CNOT RY_t(t/2)
    void cu3(int c, int t, Ang th, Ang ph, Ang la) {
        put(SV_GATE_CPHASE, c, t, la);
        put(SV_GATE_RY, t, -1, th.times(0.5));
        put(SV_GATE_CNOT, c, t);
        put(SV_GATE_RY, t, -1, th.times(-0.5));
        put(SV_GATE_CNOT, c, t);
        put(SV_GATE_CPHASE, c, t, ph);
    }

    void lower(const sv_gate &g) {
        const int a = g.q0, b = g.q1;
        switch (g.kind) {
        case SV_GATE_CY:   // S CNOT SDG
            put(SV_GATE_SDG, b);
            put(SV_GATE_CNOT, a, b);
            put(SV_GATE_S, b);
            break;
        case SV_GATE_ISWAP:   // SWAP (S (x) S) CZ
            put(SV_GATE_CZ, a, b);
            put(SV_GATE_S, a);
            put(SV_GATE_S, b);
            put(SV_GATE_SWAP, a, b);
            break;
        case SV_GATE_DCX:
            put(SV_GATE_CNOT, a, b);
            put(SV_GATE_CNOT, b, a);
            break;
        case SV_GATE_CRZ:   // CPHASE(x) P_c(-x/2)
            put(SV_GATE_P, a, -1, angle(g).times(-0.5));
            put(SV_GATE_CPHASE, a, b, angle(g));
            break;
        case SV_GATE_RZZ: rzz(a, b, angle(g)); break;
        case SV_GATE_CU1: put(SV_GATE_CPHASE, a, b, angle(g)); break;
        case SV_GATE_CSWAP: {   // CNOT(c2 -> b) CCX(a, b -> c2) CNOT(c2 -> b)
            const int c2 = (int)g.index;
            put(SV_GATE_CNOT, c2, b);
            put(SV_GATE_CCX, a, b, (uint64_t)c2);
            put(SV_GATE_CNOT, c2, b);
            break;
        }
        case SV_GATE_SX:   // H S H
        case SV_GATE_SXDG:
            put(SV_GATE_H, a);
            put(g.kind == SV_GATE_SX ? SV_GATE_S : SV_GATE_SDG, a);
            put(SV_GATE_H, a);
            break;
        case SV_GATE_R:   // RZ(p) RX(t) RZ(-p)
            put(SV_GATE_RZ, a, -1, angle(g, 1).times(-1.0));
            put(SV_GATE_RX, a, -1, angle(g, 0));
            put(SV_GATE_RZ, a, -1, angle(g, 1));
            break;
        case SV_GATE_U:   // P(p) RY(t) P(l)
            put(SV_GATE_P, a, -1, angle(g, 2));
            put(SV_GATE_RY, a, -1, angle(g, 0));
            put(SV_GATE_P, a, -1, angle(g, 1));
            break;
        case SV_GATE_RXX: rxx(a, b, angle(g)); break;
        case SV_GATE_RYY:   // (S (x) S) RXX (SDG (x) SDG)
            put(SV_GATE_SDG, a);
            put(SV_GATE_SDG, b);
            rxx(a, b, angle(g));
            put(SV_GATE_S, a);
            put(SV_GATE_S, b);
            break;
        case SV_GATE_RZX: rzx(a, b, angle(g)); break;
        case SV_GATE_ECR:   // RZX(-pi/4) X_a RZX(pi/4)
            rzx(a, b, fixed(0.25 * kPi));
            put(SV_GATE_X, a);
            rzx(a, b, fixed(-0.25 * kPi));
            break;
        case SV_GATE_CH:   // (I (x) RY(pi/4)) CZ (I (x) RY(-pi/4))
            put(SV_GATE_RY, b, -1, fixed(-0.25 * kPi));
            put(SV_GATE_CZ, a, b);
            put(SV_GATE_RY, b, -1, fixed(0.25 * kPi));
            break;
        case SV_GATE_CSX:   // (I (x) H) CPHASE(pi/2) (I (x) H)
            put(SV_GATE_H, b);
            put(SV_GATE_CPHASE, a, b, fixed(0.5 * kPi));
            put(SV_GATE_H, b);
            break;
        case SV_GATE_CU3: cu3(a, b, angle(g, 0), angle(g, 1), angle(g, 2)); break;
        case SV_GATE_CU:   // P_c(g) controlled U
            put(SV_GATE_P, a, -1, angle(g, 3));
            cu3(a, b, angle(g, 0), angle(g, 1), angle(g, 2));
            break;
        default:
            L.gates.push_back(g);
            return;
        }
        L.changed = true;
    }
};

}  // namespace

void lower_gates(const sv_gate *g, size_t n, size_t n_params, Lowering &out) {
    out.gates.clear();
    out.src.clear();
    out.scale.clear();
    out.changed = false;
    out.gates.reserve(n);
    Lowerer lw{n_params, out};
    for (size_t i = 0; i < n; ++i) lw.lower(g[i]);
}

void lower_params(const Lowering &L, const double *params, size_t n_params, int batch,
                  std::vector<double> &out) {
    out.clear();
    if (L.src.empty()) return;
    const size_t w = n_params + L.src.size();
    out.resize((size_t)batch * w);
    for (int b = 0; b < batch; ++b) {
        const double *row = params + (size_t)b * n_params;
        double *dst = out.data() + (size_t)b * w;
        for (size_t p = 0; p < n_params; ++p) dst[p] = row[p];
        for (size_t i = 0; i < L.src.size(); ++i) dst[n_params + i] = row[L.src[i]] * L.scale[i];
    }
}

}  // namespace sv
