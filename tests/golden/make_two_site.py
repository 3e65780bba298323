"""Write two_site.json: log det M, G and the force of the two-site system
K = [[0, 1], [1, 0]] from the closed form of the oracle (2 x 2 algebra written
out, exp(dk K) = cosh(dk) 1 + sinh(dk) K), for fixed fields; with them the
time-displaced G(t, t0) of every pair (from the rows of the block fermion
matrix), log det and G with the degree-4 Taylor slices of Sec. 8, and the
per-slice responses tr((1 - G~_t) A) to one fixed operator A.

    python tests/golden/make_two_site.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.closed_form import (  # noqa: E402
    two_site, two_site_displaced, two_site_slice_response, two_site_taylor)

# the operator of the stored responses
A_OP = [[0.3, 1.2 - 0.4j], [-0.7j, 2.0]]


def cpx(z):
    return [z.real, z.imag]

CASES = [
    # three slices, fields chosen by hand
    {"dk": 0.5, "phi": [[0.3, -0.7], [1.1, 0.2], [-0.4, 0.9]]},
    # twelve slices at a larger slice width (beta = 9, P = B_12 ... B_1 has
    # singular values near e^{+-9}): the stabilised path combines several QR
    # intervals
    {"dk": 0.75, "phi": [[0.1 * ((7 * t + 3 * x) % 11) - 0.5, 0.05 * ((5 * t + x) % 13) - 0.3]
                         for t in range(12) for x in (0,)]},
]


def main():
    out = []
    for case in CASES:
        ld, G, F = two_site(case["dk"], case["phi"])
        nt = len(case["phi"])
        disp = []
        for t in range(1, nt + 1):
            for t0 in range(1, nt + 1):
                Gd = two_site_displaced(case["dk"], case["phi"], t, t0)
                disp.append({"t": t, "t0": t0, "G": [[cpx(z) for z in row] for row in Gd]})
        lt, Gt = two_site_taylor(case["dk"], case["phi"], 4)
        tr = two_site_slice_response(case["dk"], case["phi"], A_OP)
        out.append({
            "dk": case["dk"],
            "phi": case["phi"],
            "logdet": [ld.real, ld.imag],
            "G": [[[z.real, z.imag] for z in row] for row in G],
            "F": [[[z.real, z.imag] for z in row] for row in F],
            "displaced": disp,
            "taylor4": {"logdet": cpx(lt), "G": [[cpx(z) for z in row] for row in Gt]},
            "response": {"A": [[cpx(complex(z)) for z in row] for row in A_OP],
                         "traces": [cpx(z) for z in tr]},
        })
    doc = {
        "source": "oracle.closed_form two_site*: K = [[0, 1], [1, 0]], "
                  "M = 1 + B_Nt ... B_1 (Sec. 2), G = M^-1, "
                  "F_{t,x} = i (1 - G~_t)_{xx} (Sec. 4 response formula), "
                  "G(t, t0) = block (t, t0) of the block inverse, propagated from G~_t0 by the "
                  "block rows; taylor4: slices with the degree-4 Taylor polynomial of exp(dk K) "
                  "(Sec. 8); response: tr((1 - G~_t) A) per slice (Sec. 4 shortcut)",
        "cases": out,
    }
    with open(os.path.join(HERE, "two_site.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
