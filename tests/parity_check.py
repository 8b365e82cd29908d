"""Comparison of per-candidate losses and gradients from the HIP path with the
FP64 oracle, where FP32 rounding may decide a discrete choice differently.

Choices of the step that depend on a comparison FP32 can decide either way
when the FP64 value lies within rounding of the threshold:
  * the side of the activation d = -eps (eps = 5e-3 dt v0, the contact
    tolerance: whether the constraint C = max(0, -d) is active, which sets
    the averaging count and the derivative rule: full or leaky);
  * the cell of a coordinate that lies on a cell face (the value is
    continuous there, the trilinear gradient is the other cell's);
  * with friction, the side of the friction cone (static or kinetic) and of
    the friction floor (a slide up to 1e-3 dt v0 gets no friction);
  * on a mesh, the side of the flat surface (the sign of the Phong distance),
    near the medial axis which of two nearly equidistant points of the
    surface is the closest, and the region (face interior, edge, vertex) of a
    closest point near a region's border.
Every reading of such a sample are correct FP32 results of the method. The
oracle reports the samples within kink_d of d = 0 and within kink_face cell
units of a face (oracle_step_ex); a candidate that misses the tolerance on
the oracle's own reading is compared again with every combination of the
other readings of its most ambiguous samples (nearest to the decision
first). It passes if one combination meets the tolerance; it is set aside
(reported, capped) only when it has more ambiguous units than are
enumerated; otherwise it fails.

FP32 error model behind the two bands:
  * contact positions come out of a chain of at most 9 rigid transforms in
    FP32; their error stays below 1e-5 of max(|p|, 1 cm) (the FK tolerance),
    about 1e-7 m here, so d = phi - r moves by about the same: a sample with
    d within KINK_D = 2.5e-7 m of -eps may land on either side;
  * a grid coordinate u = (r - lo)/h in FP32 carries the position error over
    h (1-2 mm): about 1e-4 cell units. KINK_FACE = 2e-4 cell units covers it.
Face readings of a coordinate that the seven tests share (an axis the test
does not move along, at the first iteration, where the object has not
turned) are one decision in FP32 and are flipped together.
"""
from __future__ import annotations

import itertools

import numpy as np

import oracle as O

KINK_D = 2.5e-7      # metres
KINK_FACE = 2e-4     # cell units
# tests that do not move along axis a (their first-iteration coordinate on
# that axis is the hand point's own, bit for bit in FP32)
SHARED = {1: (2, 3, 4, 5, 6), 2: (0, 1, 4, 5, 6), 3: (0, 1, 2, 3, 6)}


def units_of(amb, shared=True, kink_d=KINK_D, kink_face=KINK_FACE):
    """Independent FP32 decisions among a candidate's ambiguous samples:
    (margin relative to its band, [flip (m, k, i, what)]). The activation,
    friction and mesh decisions of samples that correct the pose come first (a
    flip changes which derivative rule or correction applies, a large change
    of the gradient); then a mesh's other nearest point for samples that only
    leak; cell-face decisions last (the value is continuous there and the
    gradient changes by the grid's second differences); each tier most
    ambiguous first. shared: the
    averaged projection, whose first iteration samples every test at the
    predicted, unturned pose (in the Gauss-Seidel sweep each constraint sees
    the pose the previous ones left, so no coordinate is shared)."""
    units = {}
    for (m, k, i, what, margin, pen) in amb:
        rel = margin / (kink_face if what in SHARED else kink_d)
        # tiers: decisions that change a correction; a mesh sample's other
        # nearest point when the sample only leaks (its normal turns by the
        # points' separation over the distance); cell faces
        tier = 2 if what in SHARED else (1 if what in (7, 8) and not pen else 0)
        if shared and what in SHARED and k == 0 and m in SHARED[what]:
            key = ("shared", i, what)
            fl = [(mm, 0, i, what) for mm in SHARED[what]]
        else:
            key = (m, k, i, what)
            fl = [(m, k, i, what)]
        if key not in units or (tier, rel) < units[key][:2]:
            units[key] = (tier, rel, fl)
    order = sorted(units.values(), key=lambda u: (u[0], u[1]))
    return [(rel, fl) for _tier, rel, fl in order]


def compare(gpu_loss, gpu_grad, H, ob, op, q, *, ltol=1e-4, gtol=1e-3, loss_floor=None, max_units=6,
            gtol_per=None, kink_d=KINK_D, kink_face=KINK_FACE, shared=None, conditioning=False, cond_cap=1e-2,
            drift=None, greedy=4, label="", say=print):
    """Checks every candidate; returns a report dict. gpu_grad may be None
    (loss only). gtol_per: optional per-candidate gradient tolerance (must be
    >= gtol).

    A candidate that misses the tolerance on the oracle's own reading is
    compared again under the other readings of its most ambiguous decisions
    (status 1 when one meets the tolerance). Without `conditioning` it is set
    aside (status 2) when it holds more ambiguous decisions than max_units
    and fails (status 3) otherwise.

    With `conditioning` (several projection iterations, where rounding early
    in the trajectory can move the later active sets) every miss is measured
    for the conditioning of the FP64 result itself: how far the oracle's loss
    and gradient move when q changes at FP32 resolution (`conditioning`). It
    passes (status 4) when both errors are within four times those movements
    and the gradient's is at most cond_cap; it is set aside as not determined
    at FP32 resolution (status 2) when the movements cover the errors but
    exceed the cap; otherwise it fails, however many ambiguous decisions it
    holds.

    drift = (kink_d, kink_face): wider bands for a form whose FP32 state
    drifts from FP64 inside the step (the Gauss-Seidel sweep, whose pose
    carries every earlier constraint's rounding). A candidate that no
    combination in the narrow bands resolves is then searched greedily over
    the decisions inside the wide bands: up to `greedy` times the reading
    that brings the result closest is added; it passes (status 5) when the
    readings found meet the tolerance."""
    q = np.asarray(q, np.float64)
    B = q.shape[0]
    if shared is None:
        shared = op.projection == 0
    want_grad = gpu_grad is not None
    ref = O.step_ex(H, ob, op, q, kink_d=kink_d, kink_face=kink_face, max_amb=256, grad=want_grad)
    floor = loss_floor if loss_floor is not None else op.w_stable * op.v0
    gt = np.full(B, gtol) if gtol_per is None else np.maximum(np.asarray(gtol_per, np.float64), gtol)

    def errs(loss_ref, grad_ref, gl, gg):
        le = abs(gl - loss_ref) / max(abs(loss_ref), floor)
        if gg is None:
            return le, 0.0
        return le, np.abs(gg - grad_ref).max() / max(np.abs(grad_ref).max(), 1e-30)

    def under(b, flip_sets):
        """(loss err, grad err) of candidate b under each set of readings."""
        gg = None if gpu_grad is None else gpu_grad[b]
        flips = [(row, *f) for row, fs in enumerate(flip_sets) for f in fs]
        alt = O.step_ex(H, ob, op, np.repeat(q[b:b + 1], len(flip_sets), axis=0), flips=flips, grad=want_grad)
        return [errs(alt["loss"][r], None if gg is None else alt["grad"][r], gpu_loss[b], gg)
                for r in range(len(flip_sets))]

    def enumerate_readings(b, cand, n_all):
        # every combination of the other readings of the most ambiguous decisions
        say(f"  {label}: candidate {b} (loss rel err {lerr[b]:.2e}, grad rel err {gerr[b]:.2e}): trying the "
            f"other readings of {len(cand)} of its {n_all} ambiguous decisions")
        subsets = [s for r in range(1, len(cand) + 1) for s in itertools.combinations(range(len(cand)), r)]
        for le, ge in under(b, [[f for u in s for f in cand[u][1]] for s in subsets]):
            if le <= ltol and ge <= gt[b]:
                return le, ge
        return None

    def greedy_readings(b):
        # readings inside the drift bands, added one at a time, closest first
        wide = O.step_ex(H, ob, op, q[b:b + 1], kink_d=drift[0], kink_face=drift[1], max_amb=1 << 14, grad=False)
        units = units_of(wide["amb"][0], shared, drift[0], drift[1])
        say(f"  {label}: candidate {b}: greedy search over {len(units)} decisions in the drift bands")
        chosen = []
        for _ in range(greedy):
            rest = [u for u in range(len(units)) if u not in chosen]
            if not rest:
                break
            res = under(b, [[f for c in chosen + [u] for f in units[c][1]] for u in rest])
            score = [max(le / ltol, ge / gt[b]) for le, ge in res]
            k = int(np.argmin(score))
            chosen.append(rest[k])
            if score[k] <= 1.0:
                return res[k]
        return None

    # 0 direct, 1 resolved by a reading, 2 set aside, 3 failed, 4 within conditioning,
    # 5 resolved by readings in the drift bands
    status = np.zeros(B, np.int32)
    lerr = np.zeros(B)
    gerr = np.zeros(B)
    n_units = np.asarray(ref["n_amb"])
    for b in range(B):
        gg = None if gpu_grad is None else gpu_grad[b]
        lerr[b], gerr[b] = errs(ref["loss"][b], None if gg is None else ref["grad"][b], gpu_loss[b], gg)
    miss = ~((lerr <= ltol) & (gerr <= gt))
    lcond = np.zeros(B)
    gcond = np.zeros(B)
    if conditioning and miss.any():
        idx = np.nonzero(miss)[0]
        lcond[idx], gcond[idx] = conditioning_of(H, ob, op, q[idx], floor=floor, grad=want_grad)
        for b in idx:
            if (lerr[b] <= max(ltol, 4.0 * lcond[b]) and gerr[b] <= max(gt[b], 4.0 * gcond[b])
                    and 4.0 * gcond[b] <= cond_cap):
                status[b] = 4
    for b in np.nonzero(miss & (status != 4))[0]:
        amb_b = ref["amb"][b]
        if ref["n_amb"][b] > len(amb_b):  # the full report of this candidate
            amb_b = O.step_ex(H, ob, op, q[b:b + 1], kink_d=kink_d, kink_face=kink_face,
                              max_amb=int(ref["n_amb"][b]), grad=False)["amb"][0]
        units = units_of(amb_b, shared, kink_d, kink_face)
        best = enumerate_readings(b, units[:max_units], len(units)) if units else None
        if best is not None:
            status[b] = 1
            lerr[b], gerr[b] = best
            continue
        if drift is not None:
            best = greedy_readings(b)
            if best is not None:
                status[b] = 5
                lerr[b], gerr[b] = best
                continue
        if conditioning:
            covered = lerr[b] <= max(ltol, 4.0 * lcond[b]) and gerr[b] <= max(gt[b], 4.0 * gcond[b])
            status[b] = 2 if covered else 3
        else:
            status[b] = 2 if len(units) > max_units else 3
    ok = (status <= 1) | (status == 5)
    rep = {"B": B, "direct": int((status == 0).sum()), "resolved": int((status == 1).sum()),
           "drift_resolved": int((status == 5).sum()),
           "conditioned": int((status == 4).sum()), "max_cond": float(gcond.max(initial=0.0)),
           "max_lcond": float(lcond.max(initial=0.0)),
           "set_aside": int((status == 2).sum()), "failed": int((status == 3).sum()),
           "max_lerr": float(lerr[ok].max(initial=0.0)),
           "max_gerr": float(gerr[ok].max(initial=0.0)),
           "ambiguous": int((n_units > 0).sum()), "status": status, "lerr": lerr, "gerr": gerr,
           "lcond": lcond, "gcond": gcond, "ref": ref}
    drift_note = f" (in the drift bands {rep['drift_resolved']})" if drift is not None else ""
    say(f"{label}: B={B} direct {rep['direct']}, resolved by an FP32 reading {rep['resolved']}{drift_note}, within "
        f"the conditioning {rep['conditioned']} (largest gradient movement {rep['max_cond']:.1e}, loss "
        f"{rep['max_lcond']:.1e}), set aside {rep['set_aside']}, failed {rep['failed']} (candidates with "
        f"ambiguous samples {rep['ambiguous']}); max loss rel err {rep['max_lerr']:.2e}, max grad rel err "
        f"(direct, resolved) {rep['max_gerr']:.2e}")
    for b in np.nonzero((status >= 2) & (status != 5))[0]:
        kind = {2: "set aside", 3: "FAILED", 4: "within conditioning"}[int(status[b])]
        say(f"  {label}: candidate {b} {kind}: loss rel err {lerr[b]:.2e} (movement {lcond[b]:.1e}), grad rel "
            f"err {gerr[b]:.2e} (movement {gcond[b]:.1e})")
    return rep


def assert_ok(rep, max_set_aside=0.01):
    bad = np.nonzero(rep["status"] == 3)[0]
    assert bad.size == 0, ("failed candidates", bad, rep["lerr"][bad], rep["gerr"][bad])
    assert rep["set_aside"] <= max_set_aside * rep["B"], ("set aside", rep["set_aside"], rep["B"])


def conditioning_of(H, ob, op, q, n=3, seed=1, floor=None, grad=True):
    """(loss movement, gradient movement) per candidate: `conditioning`."""
    return conditioning(H, ob, op, q, n=n, seed=seed, floor=floor, grad=grad)


def conditioning(H, ob, op, q, n=3, seed=1, floor=None, grad=True):
    """How far the FP64 loss and gradient move when q changes at FP32
    resolution (2^-24 relative): per candidate, the largest of n perturbed
    evaluations, the loss relative to max(|L|, floor) (floor w_s v0 by
    default) and the gradient relative to its largest component."""
    q = np.asarray(q, np.float64)
    floor = op.w_stable * op.v0 if floor is None else floor
    r0 = O.step(H, ob, op, q, grad=grad)
    lscale = np.maximum(np.abs(r0["loss"]), floor)
    gscale = np.maximum(np.abs(r0["grad"]).max(axis=1), 1e-30) if grad else None
    lc = np.zeros(q.shape[0])
    gc = np.zeros(q.shape[0])
    rng = np.random.default_rng(seed)
    for _ in range(n):
        qp = q * (1.0 + rng.normal(size=q.shape) * 6e-8)
        rp = O.step(H, ob, op, qp, grad=grad)
        lc = np.maximum(lc, np.abs(rp["loss"] - r0["loss"]) / lscale)
        if grad:
            gc = np.maximum(gc, np.abs(rp["grad"] - r0["grad"]).max(axis=1) / gscale)
    return lc, gc


def near_tie_groups(loss, tol):
    """Group ids of candidates whose sorted losses chain within tol (FP64
    losses; ties by index as the stable sort takes them)."""
    order = np.argsort(loss, kind="stable")
    gid = np.zeros(len(loss), np.int64)
    g = 0
    for k in range(1, len(order)):
        if not abs(loss[order[k]] - loss[order[k - 1]]) <= tol:
            g += 1
        gid[order[k]] = g
    return order, gid


def assert_rank_matches(rank_gpu, loss_oracle, rel=2e-4, label="", say=print):
    """The GPU's ranking is the oracle's stable sort of its FP64 losses, up
    to swaps inside groups of near-tied losses (|dL| <= rel * max |L|)."""
    loss_oracle = np.asarray(loss_oracle, np.float64)
    tol = rel * np.abs(loss_oracle).max()
    order, gid = near_tie_groups(loss_oracle, tol)
    rank_gpu = np.asarray(rank_gpu)
    assert sorted(rank_gpu.tolist()) == list(range(len(loss_oracle)))
    pos_group = gid[order]          # group of the k-th place in the oracle's order
    got_group = gid[rank_gpu]       # group of the candidate the GPU put there
    exact = int((rank_gpu == order).sum())
    say(f"{label}: ranking of {len(order)}: {exact} places identical, "
        f"{len(order) - exact} inside near-tie groups, {int(gid.max()) + 1} groups")
    assert np.array_equal(pos_group, got_group), np.nonzero(pos_group != got_group)[0][:10]
