"""Write tie_pins.json: trial DMs whose binary64 delay product lands exactly on
a half-integer, and on the double just below one, so that the delay table's
rounding rule is pinned at the tie itself.

The delay of channel c for trial DM is x = DM * k_c with
k_c = 4148.808 * (1/f_c^2 - 1/f_top^2) / tsamp and f_c = f_top - c*df (the
dispersion law of the paper's section "Searching for radio transients",
evaluated in binary64 in that order, no fused multiply-add).  Rounding is half
up: floor(x) + (x - floor(x) >= 0.5).  So

* x == n + 1/2 exactly must give n + 1 (half-to-even would give n for even n);
* x == the largest double below n + 1/2 must give n (floor(x + 1/2) gives 1
  instead of 0 for n = 0, because 0.5 + that double rounds up to 1.0).

The search walks DM through consecutive binary64 values around the target
and keeps the first whose product, computed exactly with rationals and then
rounded once to binary64 (what a single IEEE multiply does), equals the target.
Plain Python floats and fractions only; nothing here calls the oracle or the
library.  Run from the repository root:  python tests/golden/make_tie_pins.py
"""
import json
import math
import os
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))

# Bands of the synthetic workloads (LOFAR-shaped and MeerKAT-shaped).
BANDS = {
    "lofar": {"nchans": 496, "f_top": 150.0, "df": 0.1953125, "tsamp": 0.00032768},
    "meerkat": {"nchans": 4096, "f_top": 1712.0, "df": 0.104492, "tsamp": 64e-6},
}


def k_of(b, c):
    f = b["f_top"] - float(c) * b["df"]
    return 4148.808 * (1.0 / (f * f) - 1.0 / (b["f_top"] * b["f_top"])) / b["tsamp"]


def product(dm, k):
    # one IEEE binary64 multiply: exact product rounded to nearest even
    p = Fraction(dm) * Fraction(k)
    return float(p)  # Fraction -> float rounds correctly (to nearest, ties to even)


def find_dm(k, target, span=4096):
    dm0 = target / k
    lo = dm0
    for _ in range(span):
        lo = math.nextafter(lo, 0.0)
    dm = lo
    for _ in range(2 * span):
        if product(dm, k) == target:
            return dm
        dm = math.nextafter(dm, math.inf)
    return None


def main():
    cases = []
    # exact ties: n + 1/2 for even and odd n, small and large
    plan = [("lofar", 1, 0), ("lofar", 1, 3), ("lofar", 17, 6), ("lofar", 17, 41), ("lofar", 200, 1000),
            ("lofar", 200, 1001), ("lofar", 495, 86432), ("lofar", 495, 86433),
            ("meerkat", 2048, 10), ("meerkat", 2048, 11), ("meerkat", 4095, 34000), ("meerkat", 4095, 34001)]
    for band, c, n in plan:
        k = k_of(BANDS[band], c)
        for kind, target, want in (("tie", n + 0.5, n + 1),
                                   ("below", math.nextafter(n + 0.5, 0.0), n)):
            dm = find_dm(k, target)
            if dm is None:
                continue
            assert product(dm, k) == target and dm * k == target
            cases.append({"band": band, "channel": c, "dm": dm.hex(), "dm_repr": repr(dm), "kind": kind,
                          "x": target.hex(), "x_repr": repr(target), "value": want})
    doc = {
        "_about": ("Trial DMs whose binary64 delay product DM*k_c is exactly n + 1/2 ('tie', pins round half "
                   "up: value n + 1) or the largest double below n + 1/2 ('below': value n).  Delay law of the "
                   "section 'Searching for radio transients' in binary64, f_c = f_top - c*df.  Written by "
                   "tests/golden/make_tie_pins.py (plain Python floats and fractions)."),
        "bands": BANDS,
        "cases": cases,
    }
    with open(os.path.join(HERE, "tie_pins.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
        fh.write("\n")
    print("%d cases (%d ties, %d below)" % (len(cases), sum(c["kind"] == "tie" for c in cases),
                                            sum(c["kind"] == "below" for c in cases)))


if __name__ == "__main__":
    main()
