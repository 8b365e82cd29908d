"""Writes oracle_tiny.txt: the FP64 oracle's loss, loss terms and gradient on
candidates of the tiny workload (3x3 hand, 512 contacts, 64^3 sphere grid,
seeded inputs from the synthetic generators), for one and for three projection
iterations. Only the oracle computes the stored values.

Candidates are kept when every sample lies at least 1e-6 m from the
activation d = -eps (the contact tolerance) and the FP64 gradient moves by
less than 2.5e-4 of its norm under FP32-resolution changes of q, so the FP32 kernels can be held to the parity tolerances there.
Parameters and configurations are stored as FP32 values (what the kernels
receive). Rerun after any change to the oracle's arithmetic; the commit then
names the passage that justifies the change."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2306_08132_amd import synth as S  # noqa: E402

OUT = os.path.join(HERE, "oracle_tiny.txt")
N_KEEP = 8


def f32(x):
    return float(np.float32(x))


def cases():
    hand, grid, q = S.config_workload("tiny")
    H, ob = O.Hand(hand.rounded()), O.Obj(grid)
    q32 = np.asarray(q, np.float32).astype(np.float64)
    for K in (1, 3):
        prm = O.Params()
        for k in vars(prm):
            v = getattr(prm, k)
            setattr(prm, k, f32(v) if isinstance(v, float) else v)
        prm.K = K
        prm.r_dil = f32(0.005)
        ref = O.step(H, ob, prm, q32, grad=True, margins=True)
        scale = np.maximum(np.abs(ref["grad"]).max(axis=1), 1e-30)
        cond = np.zeros(q32.shape[0])
        rng = np.random.default_rng(1)
        for _ in range(3):
            qp = q32 * (1.0 + rng.normal(size=q32.shape) * 6e-8)
            cond = np.maximum(cond, np.abs(O.step(H, ob, prm, qp)["grad"] - ref["grad"]).max(axis=1) / scale)
        keep = np.nonzero((ref["min_abs_d"] > 1e-6) & (cond < 2.5e-4))[0][:N_KEEP]
        yield prm, q32[keep], ref["loss"][keep], ref["terms"][keep], ref["grad"][keep], keep


def main():
    lines = ["# Written by make_oracle_tiny.py from the FP64 oracle; do not edit by hand.",
             "# case <K> <r_dil> <n>, then per candidate: index, q (FP32 values), loss, terms, grad"]
    for prm, q, loss, terms, grad, keep in cases():
        lines.append(f"case {prm.K} {prm.r_dil:.9g} {len(keep)}")
        for i in range(len(keep)):
            lines.append(f"index {keep[i]}")
            lines.append("q " + " ".join(f"{v:.9g}" for v in q[i]))
            lines.append(f"loss {loss[i]:.17g}")
            lines.append("terms " + " ".join(f"{v:.17g}" for v in terms[i]))
            lines.append("grad " + " ".join(f"{v:.17g}" for v in grad[i]))
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
