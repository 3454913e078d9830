"""Extract the transform tables the paper prints into a JSON fixture.

Run once, on a machine that has the paper's LaTeX source, with that file's
path as the only argument:

    python tests/golden/extract_paper_tables.py PATH_TO_THE_PAPER_SOURCE

It parses, term by term, the formulas printed in
  eq. 1a-c (velocity set), eq. 59 (S), eq. 61 (S^-1),
  App. A (P f), App. B (S), App. C (F, raw -> central), App. D (B^-1
  segregation), App. E (F^-1, central -> raw), App. F (S^-1), App. G (P^-1)
and writes ``paper_appendices.json`` beside this script.  The tests compare
the oracle's matrices with these tables; nothing at run time reads the paper.

A handful of printed terms are garbled.  Each one is repaired only where the
paper's own rules fix the repair, and every repair is recorded in the
fixture's "errata" list with that rule:
  * App. C, k_202: one term lacks its operator; the binomial expansion of
    eq. 3a gives every u_x^2 u_z^2 k'_000 term the sign +.
  * App. C, k_211 and App. E, k~'_211: a central moment k_011 appears among
    raw moments; the expansion of eq. 3a (resp. App. E's rule of swapping
    k and k') only involves raw (resp. central) moments of lower order.
  * App. E, k~'_121: App. E is App. C with u -> -u; the App. C term
    -u_x u_y^2 k'_001 (odd power of u) therefore flips to +.
  * App. G, f~_4: f_3 and f_4 are mirror images in y, so f~_4 must be f~_3
    with the odd-in-y moments negated (the pair f~_1, f~_2 shows the same
    pattern in x); the printed row matches that once its leading minus sign
    is read as belonging to the first term only.
"""

import json
import os
import re
import sys


def _block(text, start_marker, end_marker):
    i = text.index(start_marker)
    j = text.index(end_marker, i + len(start_marker))
    return text[i + len(start_marker):j]


def _clean(s):
    s = s.replace("\n", " ")
    for tok in ("\\\\", "&", "\\quad", "\\;", "\\,", "\\nonumber", "\\vspace{-2em}",
                "\\begin{align*}", "\\end{align*}", "\\[", "\\]", "[4pt]", "\\!"):
        s = s.replace(tok, " ")
    return s


# ------------------------------------------------------------------ eq. 1
def parse_eq1(text):
    out = {}
    for comp in ("x", "y", "z"):
        m = re.search(r"\\ket\{e_\{" + comp + r"\}\} &=& \(([^)]*)\)\^\\dag", text)
        out[comp] = [t.strip() for t in m.group(1).split(",")]
    return out


# ------------------------------------------------------------------ scalings
def _power_pair(tok):
    """'r^2 s' -> (2, 1); 'r^{-1} s^{-2}' -> (-1, -2); '1' -> (0, 0)."""
    tok = tok.replace("{", "").replace("}", "").strip()
    pr = ps = 0
    for m in re.finditer(r"([rs])(?:\^(-?\d+))?", tok):
        e = int(m.group(2)) if m.group(2) else 1
        if m.group(1) == "r":
            pr += e
        else:
            ps += e
    return [pr, ps]


def parse_diag(text, label):
    i = text.index(label)
    seg = text[i:i + 1200]
    m = re.search(r"\\mbox\{diag\}\\big\((.*?)\\big\)", seg, re.S)
    body = m.group(1).replace("\\;", " ").replace("\\nonumber", " ").replace("&", " ").replace("\\\\", " ")
    return [_power_pair(t) for t in body.split(",")]


def parse_scaling_appendix(block, lhs_macro):
    out = {}
    pat = re.compile(r"\\" + lhs_macro + r"\{(\d{3})\}\s*=\s*([rs\^\{\}\-\d\s]*?)\s*\\" + lhs_macro + r"\{(\d{3})\}")
    for m in pat.finditer(_clean(block)):
        assert m.group(1) == m.group(3)
        out[m.group(1)] = _power_pair(m.group(2)) if m.group(2).strip() else [0, 0]
    return out


# ------------------------------------------------------------------ App. A and G
def parse_app_a(block):
    rows = {}
    s = _clean(block)
    parts = re.split(r"\\Kps\{(\d{3})\}\s*=", s)
    for name, body in zip(parts[1::2], parts[2::2]):
        terms = re.findall(r"([+-]?)\s*\\f\{(\d+)\}", body)
        rows[name] = [[-1 if sg == "-" else 1, int(a)] for sg, a in terms]
    return rows


def parse_app_g(block):
    rows = {}
    s = _clean(block)
    parts = re.split(r"\\df\{(\d+)\}\s*=", s)
    for name, body in zip(parts[1::2], parts[2::2]):
        pre = re.match(r"\s*(-?)\s*\\frac\{1\}\{(\d)\}", body)
        if pre:
            scale = (-1.0 if pre.group(1) == "-" else 1.0) / int(pre.group(2))
            body = body[pre.end():]
        else:
            scale = 1.0
        terms = re.findall(r"([+-]?)\s*\\dKps\{(\d{3})\}", body)
        rows[name] = {"scale": scale, "terms": [[-1 if sg == "-" else 1, mm] for sg, mm in terms]}
    return rows


# ------------------------------------------------------------------ App. C and E
_TERM = re.compile(r"([+-])?\s*(\d+)?\s*((?:\\u(?:xx|yy|zz|x|y|z)\s*)*)\\(d?)K(p?)s\{\s*(\d{3})\s*\}")


def _upow(s):
    px = py = pz = 0
    for m in re.finditer(r"\\u(xx|yy|zz|x|y|z)", s):
        t = m.group(1)
        if t == "x":
            px += 1
        elif t == "xx":
            px += 2
        elif t == "y":
            py += 1
        elif t == "yy":
            py += 2
        elif t == "z":
            pz += 1
        else:
            pz += 2
    return [px, py, pz]


def parse_binomial(block, lhs_macro):
    """Rows {mnp: [[coef, [px, py, pz], ijk, flags], ...]} of App. C / App. E."""
    s = _clean(block)
    parts = re.split(r"\\" + lhs_macro + r"\{(\d{3})\}\s*=", s)
    rows = {}
    for name, body in zip(parts[1::2], parts[2::2]):
        terms = []
        first = True
        for m in _TERM.finditer(body):
            sign, num, us, dmark, prime, ijk = m.groups()
            flags = []
            if sign is None and not first:
                flags.append("missing_operator")
            c = -1 if sign == "-" else 1
            c *= int(num) if num else 1
            terms.append([c, _upow(us), ijk, dmark + prime, flags])
            first = False
        rows[name] = terms
    return rows


# ------------------------------------------------------------------ App. D segregation
def parse_segregation(block):
    out = {}
    s = _clean(block)
    pat = re.compile(r"\\tilde\{k\}_\{(\d{3})\}\s*=\s*\\dfrac\{1\}\{(\d)\}\\left\((.*?)\\right\)")
    for m in pat.finditer(s):
        terms = re.findall(r"([+-])?\s*(\d)?\s*\\tilde\{k\}_\{(\w+)\}", m.group(3))
        out[m.group(1)] = {"scale": 1.0 / int(m.group(2)),
                           "terms": [[(-1 if sg == "-" else 1) * (int(n) if n else 1), name]
                                     for sg, n, name in terms]}
    return out


def main(path):
    text = open(path, encoding="utf-8").read()
    app = {}
    for k in range(1, 8):
        start = "\\label{sec:appendix%d}" % k
        nxt = "\\label{sec:appendix%d}" % (k + 1) if k < 7 else "\\end{document}"
        app[k] = _block(text, start, nxt)

    appC = parse_binomial(app[3], "Ks")
    appE = parse_binomial(app[5], "dKps")
    appG = parse_app_g(app[7])
    errata = []

    # App. C k_202: a term without operator
    for t in appC["202"]:
        if "missing_operator" in t[4]:
            t[4].remove("missing_operator")
            errata.append({"where": "App. C, k_202", "term": t[:4],
                           "fix": "missing operator read as + (binomial expansion of eq. 3a)"})
    # App. C k_211 / App. E k~'_211: central moment among raw moments
    for row, tag, want, where in ((appC["211"], "", "p", "App. C, k_211"),
                                  (appE["211"], "", "d", "App. E, k~'_211")):
        for t in row:
            if t[2] == "011" and t[3] == tag:
                t[3] = want
                errata.append({"where": where, "term": t[:3],
                               "fix": "k_011 read as the moment of the other kind used by every other term"})
    # App. E k~'_121: sign of the u_x u_y^2 k~_001 term
    for t in appE["121"]:
        if t[2] == "001" and t[1] == [1, 2, 0] and t[0] < 0:
            t[0] = -t[0]
            errata.append({"where": "App. E, k~'_121", "term": t[:3],
                           "fix": "sign flipped: App. E is App. C with u -> -u"})
    # App. G f~_4: the overall minus sign applies only to the odd-in-y moments
    g4 = appG["4"]
    if g4["scale"] < 0:
        g4["scale"] = -g4["scale"]
        g4["terms"][0][0] = -g4["terms"][0][0]
        errata.append({"where": "App. G, f~_4",
                       "fix": "the leading minus belongs to the first term only; read that way the row "
                              "is the y mirror of f~_3 (odd-in-y moments change sign)"})

    for rows in (appC, appE):
        for name, terms in rows.items():
            for t in terms:
                assert not t[4], (name, t)
                del t[4]

    fixture = {
        "source": "arXiv:2107.14774, LaTeX source; eq. 1a-c, eq. 59, eq. 61, App. A-G",
        "eq1": parse_eq1(text),
        "eq59_S": parse_diag(text, "\\label{eq:59}"),
        "eq61_Sinv": parse_diag(text, "\\label{eq:61}"),
        "appA_Pf": parse_app_a(app[1]),
        "appB_S": parse_scaling_appendix(app[2], "Kps"),
        "appC_F": appC,
        "appD_segregation": parse_segregation(app[4]),
        "appE_Finv": appE,
        "appF_Sinv": parse_scaling_appendix(app[6], "dKps"),
        "appG_Pinv": appG,
        "errata": errata,
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_appendices.json")
    with open(out, "w") as fh:
        json.dump(fixture, fh, indent=1, sort_keys=True)
    print("wrote", out, "with", len(errata), "errata")


if __name__ == "__main__":
    if len(sys.argv) != 2:
        sys.exit("usage: extract_paper_tables.py PATH_TO_THE_PAPER_SOURCE (the paper's LaTeX source)")
    main(sys.argv[1])
