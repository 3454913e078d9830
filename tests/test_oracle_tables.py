"""Pins of the oracle's lattice algebra against the tables the paper prints.

The fixture ``golden/paper_appendices.json`` holds, term by term, eq. 1a-c,
eq. 59, eq. 61 and App. A-G as printed (written by
``golden/extract_paper_tables.py`` from the paper's LaTeX source, with the five
repairs it records).  The oracle builds its matrices from their definitions;
these tests require the two to agree exactly.
"""

import json
import math
import os

import pytest
import torch

from oracle import lattice as L
from oracle import direct as D

HERE = os.path.dirname(os.path.abspath(__file__))
FIX = json.load(open(os.path.join(HERE, "golden", "paper_appendices.json")))
DT = torch.float64


def _mname(mnp):
    return "%d%d%d" % mnp


def _parse_component(tok, r, s):
    tok = tok.strip()
    sign = -1.0 if tok.startswith("-") else 1.0
    tok = tok.lstrip("-")
    val = {"0": 0.0, "1": 1.0, "r": r, "s": s}[tok]
    return sign * val


@pytest.mark.parametrize("r,s", [(1.0, 1.0), (0.7, 0.4), (0.5, 0.25)])
def test_eq1_velocity_set(r, s):
    e = L.velocities(r, s)
    for c, comp in enumerate("xyz"):
        printed = [_parse_component(t, r, s) for t in FIX["eq1"][comp]]
        assert printed == e[:, c].tolist()


def test_velocity_set_structure():
    eb = L.ebar()
    assert len({tuple(v) for v in eb.tolist()}) == 27
    assert sorted(tuple(v) for v in eb.tolist()) == sorted(
        (a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1))
    opp = L.opposite()
    # the incoming/outgoing pairs listed for the wall in Sec. 4
    for a, b in ((3, 4), (8, 9), (7, 10), (17, 16), (15, 18), (24, 21), (23, 22), (20, 25), (19, 26)):
        assert opp[a] == b and opp[b] == a


def test_appA_is_P():
    P = L.P_matrix()
    for i, mnp in enumerate(L.MOMENTS):
        row = torch.zeros(27, dtype=DT)
        for c, a in FIX["appA_Pf"][_mname(mnp)]:
            row[a] += c
        assert torch.equal(row, P[i]), mnp


def test_appG_is_P_inverse():
    Pinv = L.P_inverse()
    assert torch.allclose(Pinv @ L.P_matrix(), torch.eye(27, dtype=DT), atol=1e-14)
    for a in range(27):
        g = FIX["appG_Pinv"][str(a)]
        row = torch.zeros(27, dtype=DT)
        for c, mm in g["terms"]:
            row[L.MIDX[tuple(int(ch) for ch in mm)]] += c * g["scale"]
        assert torch.allclose(row, Pinv[a], atol=1e-14), a


def test_appG_mirror_rows():
    """f~_{2k} is f~_{2k-1} mirrored along the axis of the pair (x for 1/2, y for 3/4, z for 5/6)."""
    for first, axis in ((1, 0), (3, 1), (5, 2)):
        a = FIX["appG_Pinv"][str(first)]
        b = FIX["appG_Pinv"][str(first + 1)]
        mirrored = sorted([c * (-1) ** int(mm[axis]), mm] for c, mm in a["terms"])
        assert a["scale"] == b["scale"]
        assert mirrored == sorted(b["terms"])


@pytest.mark.parametrize("r,s", [(0.7, 0.4), (0.5, 0.25), (1.3, 0.9)])
def test_S_matches_eq59_appB(r, s):
    S = L.S_diag(r, s)
    for i, mnp in enumerate(L.MOMENTS):
        pr, ps = FIX["eq59_S"][i]
        assert S[i].item() == pytest.approx(r ** pr * s ** ps, rel=1e-15)
        qr, qs = FIX["appB_S"][_mname(mnp)]
        assert (pr, ps) == (qr, qs)
        ir, is_ = FIX["eq61_Sinv"][i]
        assert (ir, is_) == (-pr, -ps)
        fr, fs = FIX["appF_Sinv"][_mname(mnp)]
        assert (fr, fs) == (-pr, -ps)


@pytest.mark.parametrize("r,s", [(0.7, 0.4), (0.5, 0.25)])
def test_Q_is_SP_and_T_is_BQ(r, s):
    Q = L.Q_matrix(r, s)
    assert torch.allclose(Q, L.S_diag(r, s)[:, None] * L.P_matrix(), atol=1e-15)
    T = L.T_matrix(r, s)
    assert torch.allclose(T, L.B_matrix() @ Q, atol=1e-15)


def test_B_inverse_is_appD_segregation():
    Binv = L.B_inverse()
    assert torch.allclose(Binv @ L.B_matrix(), torch.eye(27, dtype=DT), atol=1e-14)
    names = {"2d1": L.N_2D1, "2d2": L.N_2D2, "2s": L.N_2S, "3s1": 10, "3s2": 11, "3s3": 12,
             "3m1": 13, "3m2": 14, "3m3": 15, "4s": 17, "4d1": 18, "4d2": 19}
    seg = FIX["appD_segregation"]
    assert len(seg) == 12
    for mm, rec in seg.items():
        row = torch.zeros(27, dtype=DT)
        for c, nm in rec["terms"]:
            row[names[nm]] += c * rec["scale"]
        assert torch.allclose(row, Binv[L.MIDX[tuple(int(ch) for ch in mm)]], atol=1e-15), mm


def _eval_binomial_table(table, u, shift_sign):
    """27x27 matrix from an App. C/E table at velocity u (a 3-tuple)."""
    M = torch.zeros(27, 27, dtype=DT)
    for mnp in L.MOMENTS:
        for c, (px, py, pz), ijk, _kind in table[_mname(mnp)]:
            mon = (shift_sign * u[0]) ** px * (shift_sign * u[1]) ** py * (shift_sign * u[2]) ** pz
            M[L.MIDX[mnp], L.MIDX[tuple(int(ch) for ch in ijk)]] += c * mon
    return M


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_appC_is_F_and_appE_is_F_inverse(seed):
    g = torch.Generator().manual_seed(seed)
    u = (torch.rand(3, generator=g, dtype=DT) - 0.5) * 0.6
    F = L.frame_matrix(u[None])[0]
    Finv = L.frame_matrix_inverse(u[None])[0]
    # App. C is written with the signs of (-u) explicit, App. E with +u
    C = _eval_binomial_table(FIX["appC_F"], u.tolist(), 1.0)
    E = _eval_binomial_table(FIX["appE_Finv"], u.tolist(), 1.0)
    assert torch.allclose(C, F, atol=1e-15)
    assert torch.allclose(E, Finv, atol=1e-15)
    assert torch.allclose(F @ Finv, torch.eye(27, dtype=DT), atol=1e-14)
    # lower triangular in the MOMENTS ordering (stated at the end of Sec. 3.1)
    assert torch.equal(torch.triu(F, 1), torch.zeros_like(F))


def test_appC_term_counts():
    """Every row holds one term per raw moment below it in each index (no term dropped)."""
    for mnp in L.MOMENTS:
        want = (mnp[0] + 1) * (mnp[1] + 1) * (mnp[2] + 1)
        assert len(FIX["appC_F"][_mname(mnp)]) == want, mnp
        assert len(FIX["appE_Finv"][_mname(mnp)]) == want, mnp


@pytest.mark.parametrize("r,s", [(1.0, 1.0), (0.6, 0.35)])
def test_central_moments_definition_equals_factor_chain(r, s):
    """eq. 3a evaluated directly equals F(u) S P for every node."""
    g = torch.Generator().manual_seed(5)
    u = (torch.rand(8, 3, generator=g, dtype=DT) - 0.5) * 0.4
    M = D.central_moment_matrix(u, r, s)
    chain = L.frame_matrix(u) @ (L.S_diag(r, s)[:, None] * L.P_matrix())
    assert torch.allclose(M, chain, atol=1e-14)


def test_errata_recorded():
    where = sorted(e["where"] for e in FIX["errata"])
    assert where == sorted(["App. C, k_202", "App. C, k_211", "App. E, k~'_211",
                            "App. E, k~'_121", "App. G, f~_4"])


def test_binomial_coefficients_are_integers():
    for tab in ("appC_F", "appE_Finv"):
        for rows in FIX[tab].values():
            for c, pw, ijk, _ in rows:
                mnp_total = sum(pw)
                assert abs(c) in (1, 2, 4, 8) and mnp_total <= 6
    assert math.comb(2, 1) == 2
