"""Writes forced_limiter_states.json: small one-dimensional states (8 cells,
periodic, a stiffened liquid and two ideal gases) on which one kind of
limiter decision of Sec. 3.3 fires -- a temperature fallback, a pressure
fallback (Sec. 3.3.1), the first-order flux (Sec. 3.3.2) and the dropped
regularization flux (Sec. 3.3.2, last paragraph).

Each state is a uniform background with one or two perturbed cells, found by
a seeded random search that calls only the oracle, then rounded to three
significant digits and checked again.  Only the primitive fields are stored
(no expected value): the tests derive what they check from the method's
admissibility conditions (Eqs. PositivityReqs1-2).

    python tests/golden/make_forced_states.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from tests.forced_cases import BITS, N, build_case  # noqa: E402


def sig3(x):
    return [float("%.3g" % v) for v in x]


def decisions(o, fields):
    case = build_case(fields)
    U = o.init_state(case)
    if not np.all(np.isfinite(U)) or not all(o.admissible(U.reshape(o.nv, N)[:, i]) for i in range(N)):
        return None
    dt, g = o.compute_dt(U)
    _, _, mask = o.rhs(U, U, (0.0, 1.0, 1.0), dt, g, with_mask=True)
    return mask


def search(want, seed):
    cdi = want == "DROP"
    o = oracle.Oracle.from_case(build_case(None, cdi=cdi))
    others = 127 & ~BITS[want]
    if want in ("T", "P"):
        others &= ~BITS["FB"]
    rng = np.random.default_rng(seed)
    best = None
    for _ in range(20000):
        f = dict(phil=[float(rng.choice([0.0, 1.0, 0.5]))] * N, yA=[float(rng.uniform())] * N,
                 P=[float(rng.choice([1e5, 1e6, 1e8]))] * N, T=[float(rng.choice([300.0, 50.0, 1000.0]))] * N,
                 u=[float(rng.choice([0.0, 100.0, -100.0, 1000.0]))] * N, cdi=cdi)
        for c in rng.choice(N, size=rng.integers(1, 3), replace=False):
            w = rng.integers(0, 5)
            if w == 0:
                f["phil"][c] = float(rng.choice([0.0, 1.0, rng.uniform() ** 6]))
            elif w == 1:
                f["yA"][c] = float(rng.choice([0.0, 1.0, rng.uniform() ** 6]))
            elif w == 2:
                f["P"][c] = float(rng.choice([-3.43e8 + 10 ** rng.uniform(2, 8), 10 ** rng.uniform(3, 10)]))
            elif w == 3:
                f["T"][c] = float(10 ** rng.uniform(-2, 4))
            else:
                f["u"][c] = float(rng.uniform(-3000, 3000))
        for k in ("phil", "yA", "P", "T", "u"):
            f[k] = sig3(f[k])
        m = decisions(o, f)
        if m is None or not np.any(m & BITS[want]) or np.any(m & others):
            continue
        nf = int(np.count_nonzero(m))
        if best is None or nf < best[0]:
            best = (nf, f)
            if nf == 1:
                break
    return best[1]


# Hand-built states.  FB: a liquid-free cell (phil = 0) in a 50/50 mixture
# under a leftward flow; the reconstructed liquid density at its upwind face
# makes the high-order flux take liquid out of a cell that has none.  DROP:
# a liquid slab whose gas side is exactly liquid-free next to a 1e-12 tail
# cell; the volume-fraction floor term of the regularization velocity moves
# liquid out of the tail cell faster than it holds it.
HAND = {
    "FB": dict(phil=[0.5, 0.5, 0.5, 0.0, 0.5, 0.5, 0.5, 0.5], yA=[0.84] * N, P=[1e5] * N, T=[50.0] * N,
               u=[-100.0] * N, cdi=False),
    "DROP": dict(phil=[0.0, 0.0, 1e-12, 0.5, 1.0, 1.0, 0.5, 1e-12], yA=[0.7] * N, P=[1e5] * N, T=[300.0] * N,
                 u=[100.0] * N, cdi=True),
}


def main():
    out = {"_doc": "Forced limiter decisions (Sec. 3.3) on 8-cell periodic states; written by "
                   "make_forced_states.py, which calls only the oracle (T, P: searched; FB, DROP: "
                   "hand-built)."}
    for want, seed in (("T", 1), ("P", 1)):
        out[want] = search(want, seed)
        print(want, out[want])
    for want, f in HAND.items():
        m = decisions(oracle.Oracle.from_case(build_case(f)), f)
        assert m is not None and np.any(m & BITS[want]), (want, m)
        out[want] = f
        print(want, f, m.tolist())
    with open(os.path.join(HERE, "forced_limiter_states.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
