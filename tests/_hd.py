"""Hyper-dual numbers and an independent evaluation of the constraints and
the Lagrangian, used to pin the oracle's Jacobian and Hessian exactly.

A hyper-dual number a + b e1 + c e2 + d e1e2 (e1^2 = e2^2 = 0) carries
f(x + e1 u + e2 v) = f + f'u e1 + f'v e2 + u^T f'' v e1e2 without
truncation error, so the e1e2 part of the Lagrangian evaluated at
w + e1 e_i + e2 e_j is exactly H_ij.

The power-flow functions are written here in the bus-admittance form
P_i = v_i sum_j v_j (G_ij cos t_ij + B_ij sin t_ij) (and Q likewise), and
the branch flows from the complex power S = V conj(y (V_f - V_t)); the
oracle uses per-branch-end derivative formulas instead.
"""
from __future__ import annotations

import numpy as np


class HD:
    __slots__ = ("a", "b", "c", "d")

    def __init__(self, a, b=0.0, c=0.0, d=0.0):
        self.a, self.b, self.c, self.d = a, b, c, d

    @staticmethod
    def lift(x):
        return x if isinstance(x, HD) else HD(x)

    def __add__(self, o):
        o = HD.lift(o)
        return HD(self.a + o.a, self.b + o.b, self.c + o.c, self.d + o.d)

    __radd__ = __add__

    def __neg__(self):
        return HD(-self.a, -self.b, -self.c, -self.d)

    def __sub__(self, o):
        return self + (-HD.lift(o))

    def __rsub__(self, o):
        return HD.lift(o) - self

    def __mul__(self, o):
        o = HD.lift(o)
        return HD(self.a * o.a, self.a * o.b + self.b * o.a, self.a * o.c + self.c * o.a,
                  self.a * o.d + self.b * o.c + self.c * o.b + self.d * o.a)

    __rmul__ = __mul__


def hsin(x):
    s, c = np.sin(x.a), np.cos(x.a)
    return HD(s, c * x.b, c * x.c, c * x.d - s * x.b * x.c)


def hcos(x):
    s, c = np.sin(x.a), np.cos(x.a)
    return HD(c, -s * x.b, -s * x.c, -s * x.d - c * x.b * x.c)


def constraints_and_objective(net, var, extra):
    """var(kind, block, index) -> HD (or float) value of a primal variable.
    extra: dict with per-block multipliers.  Returns (list of (row_key, HD)
    constraint values, HD objective)."""
    nb, nl, ng = net.nb, net.nl, net.ng
    den = net.br_r ** 2 + net.br_x ** 2
    gs, bs = net.br_r / den, -net.br_x / den
    rows = []
    agc = bool(getattr(net, "agc", False))
    for k in range(net.nblk):
        st = np.ones(nl)
        if k > 0:
            st[net.outage[k - 1]] = 0.0
        # bus admittance matrix (series branches only)
        G = np.zeros((nb, nb))
        B = np.zeros((nb, nb))
        for l in range(nl):
            f, t = net.br_from[l], net.br_to[l]
            G[f, f] += st[l] * gs[l]
            G[t, t] += st[l] * gs[l]
            B[f, f] += st[l] * bs[l]
            B[t, t] += st[l] * bs[l]
            G[f, t] -= st[l] * gs[l]
            G[t, f] -= st[l] * gs[l]
            B[f, t] -= st[l] * bs[l]
            B[t, f] -= st[l] * bs[l]
        v = [var("vm", k, i) for i in range(nb)]
        th = [var("va", k, i) for i in range(nb)]
        for i in range(nb):
            P = HD(0.0)
            Q = HD(0.0)
            for j in range(nb):
                if G[i, j] == 0.0 and B[i, j] == 0.0 and i != j:
                    continue
                tij = HD.lift(th[i]) - th[j]
                cs, sn = hcos(tij), hsin(tij)
                vv = HD.lift(v[i]) * v[j]
                P = P + vv * (G[i, j] * cs + B[i, j] * sn)
                Q = Q + vv * (G[i, j] * sn - B[i, j] * cs)
            for g in range(ng):
                if net.gen_bus[g] == i:
                    # with AGC rows a contingency block has its own generation
                    P = P - var("pgk" if agc and k > 0 else "pg", k, g)
                    Q = Q - var("qg", k, g)
            rows.append((("P", k, i), P))
            rows.append((("Q", k, i), Q))
        for l in range(nl):
            f, t = int(net.br_from[l]), int(net.br_to[l])
            g_, b_ = st[l] * gs[l], st[l] * bs[l]
            for name, s_, o_ in (("Ff", f, t), ("Ft", t, f)):
                # S = V_s conj(y (V_s - V_o)) = conj(y) |V_s|^2 - conj(y) V_s conj(V_o)
                tt = HD.lift(th[s_]) - th[o_]
                vs2 = HD.lift(v[s_]) * v[s_]
                vso = HD.lift(v[s_]) * v[o_]
                cs, sn = hcos(tt), hsin(tt)
                # conj(y) = g - jb ; V_s conj(V_o) = vso (cos + j sin)
                re = g_ * vs2 - (g_ * (vso * cs) + b_ * (vso * sn))
                im = -b_ * vs2 - (g_ * (vso * sn) - b_ * (vso * cs))
                rows.append(((name, k, l), re * re + im * im))
        if net.pvpq and k > 0:
            for g in range(ng):
                i = int(net.gen_bus[g])
                nup, num = var("nup", k, g), var("num", k, g)
                sup, slo = var("sup", k, g), var("slo", k, g)
                rows.append((("LIN", k, g), HD.lift(nup) - num - var("vm", k, i) + var("vm0", k, g)))
                rows.append((("DUP", k, g), HD.lift(sup) + var("qg", k, g)))
                rows.append((("DLO", k, g), HD.lift(slo) - var("qg", k, g)))
                rows.append((("CUP", k, g), HD.lift(num) * sup))
                rows.append((("CLO", k, g), HD.lift(nup) * slo))
        if agc and k > 0:
            # eq. (droopmpec): pi+ - pi- = p^k - (p^0 + alpha Delta), the two
            # slacks (constants dropped: they do not enter derivatives) and
            # the complementarity products pi- (pmax - p^k), pi+ (p^k - pmin)
            dk = var("delta", k, 0)
            for g in range(ng):
                pip, pim = var("pip", k, g), var("pim", k, g)
                spu, spl = var("spu", k, g), var("spl", k, g)
                pk = var("pgk", k, g)
                rows.append((("ALIN", k, g), HD.lift(pip) - pim - (HD.lift(pk) - (HD.lift(var("pg", 0, g)) + net.gen_alpha[g] * dk))))
                rows.append((("ADUP", k, g), HD.lift(spu) + pk))
                rows.append((("ADLO", k, g), HD.lift(spl) - pk))
                rows.append((("ACUP", k, g), HD.lift(pim) * spu))
                rows.append((("ACLO", k, g), HD.lift(pip) * spl))
    obj = HD(0.0)
    for g in range(ng):
        p = var("pg", 0, g)
        obj = obj + net.gen_c2[g] * (HD.lift(p) * p)
    return rows, obj
