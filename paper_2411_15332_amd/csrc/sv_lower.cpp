// Host lowering of composite Table 1 gates (see sv_lower.hpp for the rules).
#include "sv_lower.hpp"

namespace sv {

namespace {

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

struct Lowerer {
    size_t n_params;
    Lowering &L;
    // An angle of `scale` times the gate's own: a fixed angle, the caller's
    // parameter itself (scale 1) or a derived column.
    void angled(int kind, int q0, int q1, const sv_gate &g, double scale) {
        if (g.param < 0) {
            L.gates.push_back(mk(kind, q0, q1, g.angle * scale));
        } else if (scale == 1.0) {
            L.gates.push_back(mk(kind, q0, q1, 0.0, g.param));
        } else {
            const int col = (int)(n_params + L.src.size());
            L.src.push_back(g.param);
            L.scale.push_back(scale);
            L.gates.push_back(mk(kind, q0, q1, 0.0, col));
        }
    }
    void lower(const sv_gate &g) {
        const int a = g.q0, b = g.q1;
        switch (g.kind) {
        case SV_GATE_CY:
            L.gates.push_back(mk(SV_GATE_SDG, b));
            L.gates.push_back(mk(SV_GATE_CNOT, a, b));
            L.gates.push_back(mk(SV_GATE_S, b));
            break;
        case SV_GATE_ISWAP:
            L.gates.push_back(mk(SV_GATE_CZ, a, b));
            L.gates.push_back(mk(SV_GATE_S, a));
            L.gates.push_back(mk(SV_GATE_S, b));
            L.gates.push_back(mk(SV_GATE_SWAP, a, b));
            break;
        case SV_GATE_DCX:
            L.gates.push_back(mk(SV_GATE_CNOT, a, b));
            L.gates.push_back(mk(SV_GATE_CNOT, b, a));
            break;
        case SV_GATE_CRZ:
            angled(SV_GATE_P, a, -1, g, -0.5);
            angled(SV_GATE_CPHASE, a, b, g, 1.0);
            break;
        case SV_GATE_RZZ:
            angled(SV_GATE_RZ, a, -1, g, 1.0);
            angled(SV_GATE_P, b, -1, g, 1.0);
            angled(SV_GATE_CPHASE, a, b, g, -2.0);
            break;
        case SV_GATE_CU1:
            angled(SV_GATE_CPHASE, a, b, g, 1.0);
            break;
        case SV_GATE_CSWAP: {
            const int c = (int)g.index;   // second exchanged qubit
            L.gates.push_back(mk(SV_GATE_CNOT, c, b));
            L.gates.push_back(mk(SV_GATE_CCX, a, b, 0.0, -1, (uint64_t)c));
            L.gates.push_back(mk(SV_GATE_CNOT, c, b));
            break;
        }
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
