"""Slow numpy emulation of the pass-plan op semantics — TEST INFRASTRUCTURE.

Executes a plan returned by ``paper_2411_15332_amd.debug_plan`` on a host
complex128 vector, following the documented meaning of each op and layout
table (register slots, thread bits, XOR-combined index and LDS-slot tables,
tile bases). It validates the host planner on the CPU, against the oracle,
before any GPU run; the GPU kernels are checked separately by the parity tests.
"""
from __future__ import annotations

import numpy as np

(OP_EXCH, OP_D1R, OP_UDN, _UNUSED4, OP_APPLYF, _UNUSED6, _UNUSED7, OP_DENSE1, OP_H, OP_X,
 OP_CXR, OP_CXU, OP_MARK, OP_SCALE, OP_CXT, OP_D1H, OP_D2Q, OP_D1HU, OP_RPERM, OP_DENSE2,
 OP_CONT, OP_DENSE1RI, OP_CCX, OP_GENP) = range(1, 25)
NO_SOURCE = 0xFF
(SOP_D1, SOP_D2, SOP_MARK, SOP_DENSE1, SOP_DENSE2, SOP_X, SOP_Y, SOP_CX, SOP_SWAP, SOP_SCALE,
 SOP_CCX) = range(1, 12)
SRC_REG, SRC_THR, SRC_TILE = 0, 1, 2
PASS_GENERATE = 1
PASS_GEN_PRODUCT = 8


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
        elif code == SOP_CCX:
            q2 = int(op["q2"])
            i0 = idx[(((idx >> q0) & 1) == 1) & (((idx >> q1) & 1) == 1) & (((idx >> q2) & 1) == 0)]
            i1 = i0 | (1 << q2)
            psi[i0], psi[i1] = psi[i1].copy(), psi[i0].copy()
        elif code == SOP_SWAP:
            a = idx[(((idx >> q0) & 1) == 1) & (((idx >> q1) & 1) == 0)]
            b = (a & ~(1 << q0)) | (1 << q1)
            psi[a], psi[b] = psi[b].copy(), psi[a].copy()
        elif code == SOP_DENSE2:
            m = _c(c, data, 16).reshape(4, 4)
            base = idx[(((idx >> q0) & 1) == 0) & (((idx >> q1) & 1) == 0)]
            ii = [base, base | (1 << q1), base | (1 << q0), base | (1 << q0) | (1 << q1)]
            x = [psi[i].copy() for i in ii]
            for r in range(4):
                psi[ii[r]] = sum(m[r, cc] * x[cc] for cc in range(4))
        else:
            raise NotImplementedError(code)
    return psi


def run_plan(plan, psi, n):
    """Apply ``plan`` to the complex128 vector ``psi`` (length 2^n) in place."""
    if plan["small"]:
        return run_small(plan, psi, n)
    R, w, k = plan["R"], plan["w"], plan["k"]
    NR, NT = 1 << R, 1 << w
    layouts = plan["layouts"]
    t_idx = np.arange(NT, dtype=np.int64)[None, :, None]
    j_idx = np.arange(NR, dtype=np.int64)[None, None, :]
    for P in plan["passes"]:
        q = [int(x) for x in P["q"][:k]]
        tiles = int(P["tiles"])
        base = np.arange(tiles, dtype=np.int64)
        for b in q:
            base = ((base >> b) << (b + 1)) | (base & ((1 << b) - 1))
        base = base[:, None, None]
        LB = int(P["layout_begin"])

        def tables(li):
            L = layouts[LB + li]
            g = np.full((1, NT, 1), int(L["goff_xor"]), dtype=np.int64)
            s = np.full((1, NT, 1), int(L["slot_xor"]), dtype=np.int64)
            for b in range(w):
                on = ((t_idx >> b) & 1).astype(bool)
                g = np.where(on, g ^ int(L["thr_goff"][b]), g)
                s = np.where(on, s ^ int(L["thr_slot"][b]), s)
            gr = np.full((1, 1, NR), int(L["reg_goff_xor"]), dtype=np.int64)
            sr = np.zeros((1, 1, NR), dtype=np.int64)
            for p in range(R):
                on = ((j_idx >> p) & 1).astype(bool)
                gr = np.where(on, gr ^ int(L["reg_goff"][p]), gr)
                sr = np.where(on, sr ^ int(L["reg_slot"][p]), sr)
            return (g, gr), s ^ sr

        def addresses(li):
            # (tile base | thread part) XOR register part: the register part
            # may carry the global XOR translation of bits off the tile
            (g, gr), _ = tables(li)
            assert np.all((g & base) == 0)
            addr = (base | g) ^ gr
            assert all(np.unique(addr[t]).size == NT * NR for t in range(min(tiles, 4)))
            return addr

        gidx = addresses(0)
        if int(P["flags"]) & PASS_GEN_PRODUCT:
            # amp[i] = prod_q u_q[bit q of i], u from the OP_GENP record and
            # its continuations (4 reals per qubit: u_q0, u_q1)
            g0 = plan["ops"][int(P["op_begin"])]
            assert int(g0["code"]) == OP_GENP
            nq, ncont = int(g0["a"]), int(g0["b"])
            recs = plan["ops"][int(P["op_begin"]): int(P["op_begin"]) + 1 + ncont]
            vals = np.concatenate([r["payload"] for r in recs])   # FP64 in both precisions
            u = (vals[0::2] + 1j * vals[1::2]).reshape(-1, 2)[:nq]
            a = np.ones(gidx.shape, dtype=np.complex128)
            for q in range(nq):
                a = a * u[q][(gidx >> q) & 1]
        elif int(P["flags"]) & PASS_GENERATE:
            gj, gm, sc = int(P["gen_j"]), int(P["gen_mask"]), float(P["gen_scale"])
            on = ((gidx ^ gj) & ~gm) == 0
            par = np.vectorize(lambda x: bin(x).count("1") & 1)(gidx & gj & gm)
            a = np.where(on, np.where(par == 1, -sc, sc), 0.0).astype(np.complex128)
        else:
            a = psi[gidx].copy()
        f = np.ones((tiles, NT, 1), dtype=np.complex128)

        def src_bit(s):
            kind, pos = s >> 6, s & 63
            if kind == SRC_THR:
                return np.broadcast_to((t_idx >> pos) & 1, (tiles, NT, 1))
            assert kind == SRC_TILE
            return np.broadcast_to((base >> pos) & 1, (tiles, NT, 1))

        def pairs(p):
            lo = [j for j in range(NR) if not (j >> p) & 1]
            return lo, [j | (1 << p) for j in lo]

        ops = plan["ops"]
        for oi in range(int(P["op_begin"]), int(P["op_end"])):
            op = ops[oi]
            code, oa, ob, sa, sb, data = (int(op["code"]), int(op["a"]), int(op["b"]),
                                          int(op["sa"]), int(op["sb"]), int(op["data"]))
            pl = op["payload"].view(np.float32).astype(np.float64) if plan.get("f32") else op["payload"]
            d = pl[0::2] + 1j * pl[1::2]
            if code == OP_EXCH:
                # the per-thread factor does not travel with the amplitudes
                assert np.all(f == 1), "pending per-thread factor at an exchange"
                # Two halves through a half-tile buffer: the half is the value
                # of label sb, taken from the same register bit or thread bit
                # (source sa) on both sides; slots drop bit sb.
                lab = sb
                assert lab >= plan["m"], "split label inside the swizzle bits"
                kind, pos = sa >> 6, sa & 63
                shape = (tiles, NT, NR)
                half = np.broadcast_to(((j_idx >> pos) & 1) if kind == SRC_REG else ((t_idx >> pos) & 1),
                                       shape)
                assert kind in (SRC_REG, SRC_THR)
                _, sw = tables(oa)
                _, sr = tables(ob)
                sw = np.broadcast_to(sw, shape)
                sr = np.broadcast_to(sr, shape)
                assert np.all(np.sort(sw[0].ravel()) == np.arange(1 << k))
                assert np.all(np.sort(sr[0].ravel()) == np.arange(1 << k))
                # the buffer half is one value of the label on both sides
                cw = ((sw >> lab) & 1) ^ half
                cr = ((sr >> lab) & 1) ^ half
                assert np.all(cw == cw.flat[0]) and np.all(cr == cw.flat[0])
                lo = (1 << lab) - 1
                cw_slot = (sw & lo) | ((sw >> 1) & ~lo)
                cr_slot = (sr & lo) | ((sr >> 1) & ~lo)
                out = np.full(shape, np.nan, dtype=np.complex128)
                for h in (0, 1):
                    lds = np.full((tiles, 1 << (k - 1)), np.nan, dtype=np.complex128)
                    wm = half == h
                    ws = cw_slot[wm].reshape(tiles, -1)
                    assert np.all(np.sort(ws[0]) == np.arange(1 << (k - 1)))
                    np.put_along_axis(lds, ws, a[wm].reshape(tiles, -1), axis=1)
                    rs = cr_slot[half == h].reshape(tiles, -1)
                    vals = np.take_along_axis(lds, rs, axis=1)
                    assert not np.any(np.isnan(vals))
                    out[half == h] = vals.ravel()
                a = out
            elif code == OP_D1R:
                a = a * f * d[:2][(j_idx >> oa) & 1]
                f = np.ones_like(f)
            elif code == OP_UDN:
                g = np.full((tiles, NT, 1), d[0], dtype=np.complex128)
                for i in range(oa):
                    if i < 4:
                        s1, s2 = (data >> (16 * i)) & 0xFF, (data >> (16 * i + 8)) & 0xFF
                    else:
                        s1, s2 = sa, sb
                    on = src_bit(s1) & (1 if s2 == NO_SOURCE else src_bit(s2))
                    g = np.where(on == 1, g * d[i + 1], g)
                f = f * g
            elif code == OP_CONT:
                continue   # payload of the preceding OP_DENSE2
            elif code == OP_RPERM:
                sel = [j for j in range(NR) if (j >> oa) & 1 and not (j >> ob) & 1]
                oth = [j ^ (1 << oa) ^ (1 << ob) for j in sel]
                a[:, :, sel], a[:, :, oth] = a[:, :, oth].copy(), a[:, :, sel].copy()
            elif code == OP_DENSE2:
                per = 8 if plan.get("f32") else 4
                ent = []
                for t in range(16 // per):
                    rec = ops[oi + t]
                    v = rec["payload"].view(np.float32).astype(np.float64) if plan.get("f32") else rec["payload"]
                    ent += list(v[0::2][:per] + 1j * v[1::2][:per])
                m = np.array(ent).reshape(4, 4)
                for j0 in range(0, NR, 4):
                    x = [a[:, :, j0 + e].copy() for e in range(4)]
                    for r in range(4):
                        a[:, :, j0 + r] = sum(m[r, cc] * x[cc] for cc in range(4))
            elif code == OP_D1H:
                sel = ((j_idx >> oa) & 1) == ob
                a = np.where(sel, a * d[0], a)
            elif code == OP_D2Q:
                sel = (((j_idx >> oa) & 1) == (sa & 1)) & (((j_idx >> ob) & 1) == ((sa >> 1) & 1))
                a = np.where(sel, a * d[0], a)
            elif code == OP_D1HU:
                sel = (((j_idx >> oa) & 1) == (ob & 1)) & (src_bit(sa) == ((ob >> 1) & 1))
                a = np.where(sel, a * d[0], a)
            elif code == OP_APPLYF:
                a = a * f
                f = np.ones_like(f)
            elif code == OP_DENSE1:
                lo, hi = pairs(oa)
                x0, x1 = a[:, :, lo], a[:, :, hi]
                if ob:
                    a[:, :, lo], a[:, :, hi] = f * (d[0] * x0 + d[1] * x1), f * (d[2] * x0 + d[3] * x1)
                    f = np.ones_like(f)
                else:
                    a[:, :, lo], a[:, :, hi] = d[0] * x0 + d[1] * x1, d[2] * x0 + d[3] * x1
            elif code == OP_DENSE1RI:
                g0, g1, bt = ob & 1, (ob >> 1) & 1, (ob >> 2) & 1
                m = np.array([[pl[0], pl[1]], [pl[2], pl[3]]], dtype=np.complex128)
                m = np.diag([1j ** g0, 1j ** g1]) @ m @ np.diag([1, 1j ** bt])
                lo, hi = pairs(oa)
                x0, x1 = a[:, :, lo], a[:, :, hi]
                a[:, :, lo], a[:, :, hi] = m[0, 0] * x0 + m[0, 1] * x1, m[1, 0] * x0 + m[1, 1] * x1
            elif code == OP_H:
                assert oa and oa < (1 << R)
                for bit in range(R):
                    if (oa >> bit) & 1:
                        lo, hi = pairs(bit)
                        x0, x1 = a[:, :, lo], a[:, :, hi]
                        a[:, :, lo], a[:, :, hi] = x0 + x1, x0 - x1
            elif code == OP_X:
                lo, hi = pairs(oa)
                a[:, :, lo], a[:, :, hi] = a[:, :, hi].copy(), a[:, :, lo].copy()
            elif code == OP_CXR:
                lo = [j for j in range(NR) if not (j >> oa) & 1 and (j >> ob) & 1]
                hi = [j | (1 << oa) for j in lo]
                a[:, :, lo], a[:, :, hi] = a[:, :, hi].copy(), a[:, :, lo].copy()
            elif code == OP_CXU:
                lo, hi = pairs(oa)
                cb = src_bit(sa).astype(bool)
                x0, x1 = a[:, :, lo], a[:, :, hi]
                a[:, :, lo], a[:, :, hi] = np.where(cb, x1, x0), np.where(cb, x0, x1)
            elif code == OP_CXT:
                lo, hi = pairs(oa)
                cb = src_bit(sa).astype(bool)
                x0, x1 = a[:, :, lo], a[:, :, hi]
                a[:, :, lo], a[:, :, hi] = np.where(cb, x1, x0), np.where(cb, x0, x1)
            elif code == OP_CCX:
                cm, cv, uv = ob, data & 0xFF, (data >> 8) & 3
                assert cv & ~cm == 0
                on = np.ones((tiles, NT, 1), dtype=bool)
                if sa != NO_SOURCE:
                    on &= src_bit(sa) == (uv & 1)
                if sb != NO_SOURCE:
                    on &= src_bit(sb) == (uv >> 1)
                lo = [j for j in range(NR) if not (j >> oa) & 1 and (j & cm) == cv]
                hi = [j | (1 << oa) for j in lo]
                x0, x1 = a[:, :, lo].copy(), a[:, :, hi].copy()
                a[:, :, lo], a[:, :, hi] = np.where(on, x1, x0), np.where(on, x0, x1)
            elif code == OP_MARK:
                hit = (base == data) & (t_idx == (sa | (sb << 8))) & (j_idx == oa)
                a = np.where(hit, -a, a)
            elif code == OP_SCALE:
                a = a * pl[0]
            elif code == OP_GENP:
                assert oi == int(P["op_begin"]), "product data outside the pass's first record"
            else:
                raise NotImplementedError(code)
        assert np.all(f == 1), "pending per-thread factor at the store"
        sidx = addresses(int(P["store_layout"]))
        # in place: every workgroup stores exactly the addresses it loaded
        assert np.array_equal(np.sort(sidx.reshape(tiles, -1), axis=1),
                              np.sort(np.broadcast_to(gidx, sidx.shape).reshape(tiles, -1), axis=1))
        psi[sidx] = a
    return psi
