// Host fuzz of gate validation, lowering and planning (no GPU), built and run
// under AddressSanitizer and UndefinedBehaviorSanitizer by test_host_sanitizers.py.
#include <cstdio>
#include <random>
#include <stdexcept>
#include <vector>
#include "sv_lower.hpp"
#include "sv_planner.hpp"
using namespace sv;
static const int kinds2q[] = {SV_GATE_CNOT, SV_GATE_CZ, SV_GATE_SWAP, SV_GATE_CPHASE, SV_GATE_U2, SV_GATE_CY,
                              SV_GATE_ISWAP, SV_GATE_DCX, SV_GATE_CRZ, SV_GATE_RZZ, SV_GATE_CU1, SV_GATE_RXX,
                              SV_GATE_RYY, SV_GATE_RZX, SV_GATE_ECR, SV_GATE_CH, SV_GATE_CSX, SV_GATE_CU3, SV_GATE_CU};
static const int kinds1q[] = {SV_GATE_I, SV_GATE_X, SV_GATE_Y, SV_GATE_Z, SV_GATE_H, SV_GATE_S, SV_GATE_SDG,
                              SV_GATE_T, SV_GATE_TDG, SV_GATE_RX, SV_GATE_RY, SV_GATE_RZ, SV_GATE_P, SV_GATE_U1,
                              SV_GATE_SX, SV_GATE_SXDG, SV_GATE_R, SV_GATE_U};
int main(int argc, char **argv) {
    const int iters = argc > 1 ? atoi(argv[1]) : 300;
    std::mt19937_64 rng(7);
    long plans = 0, ops = 0;
    for (int it = 0; it < iters; ++it) {
        const int n = 1 + (int)(rng() % 30);
        const bool c64 = rng() & 1;
        PlanOptions o;
        o.R = c64 ? 5 : 4; o.v = c64 ? 1 : 0; o.m = c64 ? 4 : 3; o.ud_max = c64 ? 5 : 3;
        o.small_max = c64 ? 13 : 12; o.w_max = 8;
        o.c = 3 + (int)(rng() % 5); o.auto_low = rng() % 3 == 0; if (o.auto_low) o.c = 6;
        o.fuse = rng() % 8 != 0; o.remap = rng() % 4 != 0; o.gen_h = rng() & 1;
        o.basis_known = rng() & 1; o.basis_j = n < 64 ? rng() % (1ull << n) : 0;
        o.small_mode = 1 + (int)(rng() % 2); o.max_dense = rng() % 5 == 0 ? 1 + (int)(rng() % 4) : 1 << 20;
        std::vector<sv_gate> g;
        std::vector<double> params;
        const int ng = (int)(rng() % 200);
        for (int i = 0; i < ng; ++i) {
            sv_gate x{};
            x.param = -1; x.q1 = -1;
            x.angle = (double)(rng() % 1000) * 0.01 - 5.0;
            const int pick = (int)(rng() % 10);
            if (pick < 5 || n < 2) {
                x.kind = kinds1q[rng() % (sizeof kinds1q / sizeof(int))];
                x.q0 = (int)(rng() % n);
            } else if (pick < 9 || n < 3) {
                x.kind = kinds2q[rng() % (sizeof kinds2q / sizeof(int))];
                x.q0 = (int)(rng() % n);
                do x.q1 = (int)(rng() % n); while (x.q1 == x.q0);
            } else if (pick == 9 && n >= 3) {
                x.kind = rng() & 1 ? SV_GATE_CCX : SV_GATE_CSWAP;
                x.q0 = (int)(rng() % n);
                do x.q1 = (int)(rng() % n); while (x.q1 == x.q0);
                int q2; do q2 = (int)(rng() % n); while (q2 == x.q0 || q2 == x.q1);
                x.index = (uint64_t)q2;
            }
            if (rng() % 10 == 0) { x.kind = SV_GATE_MARK; x.q0 = -1; x.q1 = -1; x.index = n < 64 ? rng() % (1ull << n) : 0; }
            const int need = x.kind == SV_GATE_U1 ? 8 : x.kind == SV_GATE_U2 ? 32 : x.kind == SV_GATE_R ? 2
                           : (x.kind == SV_GATE_U || x.kind == SV_GATE_CU3) ? 3 : x.kind == SV_GATE_CU ? 4 : 0;
            const bool angled = x.kind == SV_GATE_RX || x.kind == SV_GATE_RY || x.kind == SV_GATE_RZ ||
                                x.kind == SV_GATE_P || x.kind == SV_GATE_CPHASE || x.kind == SV_GATE_CRZ ||
                                x.kind == SV_GATE_RZZ || x.kind == SV_GATE_CU1 || x.kind == SV_GATE_RXX ||
                                x.kind == SV_GATE_RYY || x.kind == SV_GATE_RZX;
            if (need || (angled && rng() % 2 == 0)) {
                x.param = (int)params.size();
                for (int k = 0; k < (need ? need : 1); ++k) params.push_back((double)(rng() % 1000) * 0.001);
            }
            g.push_back(x);
        }
        std::string err;
        if (!validate_gates(n, g.data(), g.size(), params.size(), true, err)) {
            printf("invalid n=%d it=%d: %s\n", n, it, err.c_str());
            return 1;
        }
        Lowering low;
        lower_gates(g.data(), g.size(), params.size(), low);
        const int batch = 1 + (int)(rng() % 3);
        std::vector<double> table((size_t)batch * std::max<size_t>(params.size(), 1));
        for (int b = 0; b < batch; ++b) for (size_t p = 0; p < params.size(); ++p) table[b * params.size() + p] = params[p] + b;
        std::vector<double> ext;
        lower_params(low, table.data(), params.size(), batch, ext);
        const double *pp = ext.empty() ? table.data() : ext.data();
        const size_t pn = params.size() + low.src.size();
        if (n > 34) continue;
        if (n >= 31 && !o.auto_low) {}  // large n are planned too (host only)
        Plan p;
        try {
            p = build_plan_auto(n, low.gates.data(), low.gates.size(), o);
        } catch (const std::exception &e) {
            printf("EXCEPTION n=%d it=%d: %s\n", n, it, e.what());
            return 1;
        }
        ++plans;
        ops += (long)p.ops.size();
        if (p.small) {
            std::vector<double> cst((size_t)batch * std::max<uint64_t>(p.cstride, 1));
            materialize_consts(p, low.gates.data(), pp, pn, batch, c64, cst.data());
        } else if (!p.ops.empty()) {
            std::vector<DevOp> out((size_t)batch * p.ops.size());
            materialize_ops(p, low.gates.data(), pp, pn, batch, c64, out.data());
        }
    }
    printf("ok plans=%ld ops=%ld\n", plans, ops);
    return 0;
}
