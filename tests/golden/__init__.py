"""Hand-derived examples (JSON), each with the passage it follows and its
derivation.  Values are exact: rationals as "p/q" strings, logarithms as
{"log": [[coefficient, "p/q"], ...]} meaning the sum of coefficient *
log(p/q); eta given as {"log_of": [...]} means eta_m = log of each entry."""
import json
import math
import os
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))


def value(v):
    if isinstance(v, dict) and "log" in v:
        return sum(c * math.log(Fraction(q)) for c, q in v["log"])
    if isinstance(v, dict) and "log_of" in v:
        return [math.log(Fraction(q)) for q in v["log_of"]]
    if isinstance(v, list):
        return [value(x) for x in v]
    if isinstance(v, str):
        return float(Fraction(v))
    return float(v)


def load(name):
    with open(os.path.join(HERE, name + ".json")) as f:
        d = json.load(f)
    out = {k: (value(v) if k not in ("citation", "derivation", "model") else v)
           for k, v in d.items()}
    return out


NAMES = ["cox_hand", "cox_ties_hand", "fg_hand"]
