"""Algorithmic FP64 operation counts of the hot path, by the oracle's counting
scalar, on a sub-box of the benchmark workload; writes oracle/op_counts.json.

Counts + - * / sqrt log tanh once each, for one right-hand side: per face of
each sweep direction and per cell (equilibrium and auxiliaries)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from paper_2504_14063_amd import inputs  # noqa: E402


def box(case, m):
    idx = [(np.arange(m) + int(round(case.extra["center"][d])) - m // 2) % case.n[d] for d in range(3)]
    sub = lambda a: np.ascontiguousarray(a[..., idx[2], :, :][..., :, idx[1], :][..., :, :, idx[0]])
    return inputs.Case("box", 3, (m, m, m), case.dx, (0, 0, 0), (0, 0, 0), case.materials, case.opts,
                       sub(case.phi), sub(case.y), sub(case.P), sub(case.T), sub(case.vel))


def main(m=40):
    case = inputs.droplet_crossflow_3d(n=256)
    b = box(case, m)
    o = oracle.Oracle.from_case(b)
    U = o.init_state(b)
    dt, g = o.compute_dt(U)
    c = o.count_ops(U, dt, g)
    faces = o.face_counts()
    res = dict(cell=c["cell"] / c["padded_cells"],
               face_x=c["face_x"] / faces[0], face_y=c["face_y"] / faces[1], face_z=c["face_z"] / faces[2],
               divergence=c["divergence"] / o.ncell)
    res["per_cell_update"] = 3 * (res["cell"] + res["face_x"] + res["face_y"] + res["face_z"]
                                  + res["divergence"])
    res["sample"] = f"{m}^3 periodic sub-box centred on the droplet of droplet_crossflow_3d 256^3"
    out = {"droplet_crossflow_3d": res}
    with open(os.path.join(HERE, "op_counts.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
