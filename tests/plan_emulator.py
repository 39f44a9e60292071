"""Slow numpy emulation of the pass-plan op semantics — TEST INFRASTRUCTURE.

Executes a plan returned by ``paper_2411_15332_amd.debug_plan`` on a host
complex128 vector, following the documented meaning of each op (register
slots, thread bits, LDS exchanges with the slot swizzle, tile bases). It
validates the host planner on the CPU, against the oracle, before any GPU run;
the GPU kernels are checked separately by the parity tests.
"""
from __future__ import annotations

import numpy as np

OP_EXCH, OP_D1, OP_D2, OP_MARK, OP_DENSE1, OP_H, OP_X, OP_Y, OP_CX, OP_SWAP, OP_DENSE2, OP_SCALE = range(1, 13)
SOP_D1, SOP_D2, SOP_MARK, SOP_DENSE1, SOP_DENSE2, SOP_X, SOP_Y, SOP_CX, SOP_SWAP, SOP_SCALE = range(1, 11)
SRC_REG, SRC_THR, SRC_TILE = 0, 1, 2
PASS_GENERATE = 1

SWZ3 = [1, 2, 4, 3, 6, 7, 5]
SWZ4 = [1, 2, 4, 8, 3, 6, 12, 11, 5, 10, 7, 14, 15, 13, 9]


def swz_image(b, m):
    if b < m:
        return 1 << b
    return SWZ3[(b - 3) % 7] if m == 3 else SWZ4[(b - 4) % 15]


def swz_slot(l, m):
    s = 0
    for b in range(m, 32):
        if (l >> b) & 1:
            s ^= swz_image(b, m)
    return l ^ s


def _c(consts, off, count):
    v = consts[off: off + 2 * count]
    return v[0::2] + 1j * v[1::2]


def run_small(plan, psi, n):
    N = 1 << n
    c = plan["consts"]
    idx = np.arange(N)
    for op in plan["sops"]:
        code, q0, q1, data = int(op["code"]), int(op["q0"]), int(op["q1"]), int(op["data"])
        if code == SOP_D1:
            d = _c(c, data, 2)
            psi *= d[(idx >> q0) & 1]
        elif code == SOP_D2:
            d = _c(c, data, 4)
            psi *= d[(((idx >> q0) & 1) << 1) | ((idx >> q1) & 1)]
        elif code == SOP_MARK:
            psi[data] = -psi[data]
        elif code in (SOP_DENSE1, SOP_X, SOP_Y):
            i0 = idx[((idx >> q0) & 1) == 0]
            i1 = i0 | (1 << q0)
            x0, x1 = psi[i0].copy(), psi[i1].copy()
            if code == SOP_DENSE1:
                g = _c(c, data, 4)
                psi[i0] = g[0] * x0 + g[1] * x1
                psi[i1] = g[2] * x0 + g[3] * x1
            elif code == SOP_X:
                psi[i0], psi[i1] = x1, x0
            else:
                psi[i0], psi[i1] = -1j * x1, 1j * x0
        elif code == SOP_CX:
            i0 = idx[(((idx >> q0) & 1) == 1) & (((idx >> q1) & 1) == 0)]
            i1 = i0 | (1 << q1)
            psi[i0], psi[i1] = psi[i1].copy(), psi[i0].copy()
        elif code == SOP_SWAP:
            a = idx[(((idx >> q0) & 1) == 1) & (((idx >> q1) & 1) == 0)]
            b = (a & ~(1 << q0)) | (1 << q1)
            psi[a], psi[b] = psi[b].copy(), psi[a].copy()
        elif code == SOP_DENSE2:
            raise NotImplementedError
        elif code == SOP_SCALE:
            psi *= c[data]
    return psi


def run_plan(plan, psi, n):
    """Apply ``plan`` to the complex128 vector ``psi`` (length 2^n) in place."""
    if plan["small"]:
        return run_small(plan, psi, n)
    R, m, w, k = plan["R"], plan["m"], plan["w"], plan["k"]
    NR, NT = 1 << R, 1 << w
    consts = plan["consts"]
    layouts = plan["layouts"]
    t_idx = np.arange(NT)[None, :, None]
    j_idx = np.arange(NR)[None, None, :]
    for P in plan["passes"]:
        q = [int(x) for x in P["q"][:k]]
        tiles = int(P["tiles"])
        tau = np.arange(tiles, dtype=np.int64)
        base = tau.copy()
        for b in q:
            base = ((base >> b) << (b + 1)) | (base & ((1 << b) - 1))
        base = base[:, None, None]

        def lay(li):
            L = layouts[int(P["layout_begin"]) + li]
            reg = [int(x) for x in L["reg_local"][:R]]
            thr = [int(x) for x in L["thr_local"][:w]]
            loc = np.zeros((1, NT, NR), dtype=np.int64)
            glob = np.zeros((1, NT, NR), dtype=np.int64)
            for s, lb in enumerate(thr):
                bit = (t_idx >> s) & 1
                loc = loc | (bit << lb)
                glob = glob | (bit << q[lb])
            for p, lb in enumerate(reg):
                bit = (j_idx >> p) & 1
                loc = loc | (bit << lb)
                glob = glob | (bit << q[lb])
            return reg, thr, loc, glob

        cur = 0
        reg, thr, loc, glob = lay(cur)
        gidx = base | glob
        if int(P["flags"]) & PASS_GENERATE:
            gj, gm, sc = int(P["gen_j"]), int(P["gen_mask"]), float(P["gen_scale"])
            on = ((gidx ^ gj) & ~gm) == 0
            par = np.vectorize(lambda x: bin(x).count("1") & 1)(gidx & gj & gm)
            a = np.where(on, np.where(par == 1, -sc, sc), 0.0).astype(np.complex128)
        else:
            a = psi[gidx]

        def src_bit(s):
            kind, pos = s >> 6, s & 63
            if kind == SRC_REG:
                return np.broadcast_to((j_idx >> pos) & 1, a.shape)
            if kind == SRC_THR:
                return np.broadcast_to((t_idx >> pos) & 1, a.shape)
            return np.broadcast_to((base >> pos) & 1, a.shape)

        for op in plan["ops"][int(P["op_begin"]): int(P["op_end"])]:
            code, oa, ob, sa, sb, data = (int(op["code"]), int(op["a"]), int(op["b"]),
                                          int(op["sa"]), int(op["sb"]), int(op["data"]))
            if code == OP_EXCH:
                lds = np.zeros((tiles, 1 << k), dtype=np.complex128)
                slots = np.vectorize(lambda l: swz_slot(int(l), m))(loc)
                np.put_along_axis(lds, np.broadcast_to(slots, a.shape).reshape(tiles, -1),
                                  a.reshape(tiles, -1), axis=1)
                cur = oa
                reg, thr, loc, glob = lay(cur)
                slots = np.vectorize(lambda l: swz_slot(int(l), m))(loc)
                a = np.take_along_axis(lds, np.broadcast_to(slots, a.shape).reshape(tiles, -1),
                                       axis=1).reshape(a.shape)
            elif code == OP_D1:
                d = _c(consts, data, 2)
                a = a * d[src_bit(sa)]
            elif code == OP_D2:
                d = _c(consts, data, 4)
                a = a * d[(src_bit(sa) << 1) | src_bit(sb)]
            elif code == OP_MARK:
                hit = (base == data) & (t_idx == ob) & (j_idx == oa)
                a = np.where(hit, -a, a)
            elif code == OP_SCALE:
                a = a * consts[data]
            else:
                p = oa
                lo = [j for j in range(NR) if not (j >> p) & 1]
                hi = [j | (1 << p) for j in lo]
                x0, x1 = a[:, :, lo], a[:, :, hi]
                if code == OP_DENSE1:
                    g = _c(consts, data, 4)
                    a[:, :, lo], a[:, :, hi] = g[0] * x0 + g[1] * x1, g[2] * x0 + g[3] * x1
                elif code == OP_H:
                    a[:, :, lo], a[:, :, hi] = x0 + x1, x0 - x1
                elif code == OP_X:
                    a[:, :, lo], a[:, :, hi] = x1, x0
                elif code == OP_Y:
                    a[:, :, lo], a[:, :, hi] = -1j * x1, 1j * x0
                elif code == OP_CX:
                    cb = src_bit(sa)[:, :, lo].astype(bool)
                    a[:, :, lo], a[:, :, hi] = np.where(cb, x1, x0), np.where(cb, x0, x1)
                elif code == OP_SWAP:
                    pa, pb = oa, ob
                    s10 = [j for j in range(NR) if (j >> pa) & 1 and not (j >> pb) & 1]
                    s01 = [(j & ~(1 << pa)) | (1 << pb) for j in s10]
                    a[:, :, s10], a[:, :, s01] = a[:, :, s01].copy(), a[:, :, s10].copy()
                else:
                    raise NotImplementedError(code)
        psi[base | glob] = a
    return psi
