"""Executes an exported transform schedule on the CPU with exact ring arithmetic.

Test infrastructure: the schedule (passes of leaf jobs, leaf programs of
base-case operations) comes from the library's host planner through
``tft_plan_export``; this module applies the base cases of Alg. 1 and Alg. 2
(L = 2) exactly as the paper states them, on cells held as Python values, so
that the planner's expansion of the recursion can be compared with the oracle
without a GPU.  Cells a leaf job does not load are replaced by fresh random
values, so a schedule that reads a cell it should not read is caught.
"""

import random

OP_NONE, OP_T22, OP_T21, OP_T12, OP_I2, OP_I1F1Z2, OP_I1F1Z1, OP_I1F0Z2, OP_I1F0Z1, OP_I0Z2, OP_I0Z1 = range(11)


def _rand(ring, rng):
    if ring.kind in ("fermat", "prime"):
        return rng.randrange(ring.p)
    return tuple(rng.randrange(ring.m) for _ in range(ring.K))


def apply_op(ring, code, x0, x1, e):
    """One base case (Alg. 1 / Alg. 2 at L = 2) with zeta = theta^e; returns (x0, x1)."""
    two = ring.add(ring.theta_pow(0), ring.theta_pow(0))
    if code == OP_T22:
        return ring.add(x0, x1), ring.mul_theta(ring.sub(x0, x1), e)
    if code == OP_T21:
        return x0, ring.mul_theta(x0, e)
    if code == OP_T12:
        return ring.add(x0, x1), x1
    if code == OP_I2:
        t = ring.mul_theta(x1, -e)
        return ring.add(x0, t), ring.sub(x0, t)
    if code == OP_I1F1Z2:
        return ring.sub(ring.mul(two, x0), x1), ring.mul_theta(ring.sub(x0, x1), e)
    if code == OP_I1F1Z1:
        return ring.mul(two, x0), ring.mul_theta(x0, e)
    if code == OP_I1F0Z2:
        return ring.sub(ring.mul(two, x0), x1), x1
    if code == OP_I1F0Z1:
        return ring.mul(two, x0), x1
    if code == OP_I0Z2:
        return ring.mul(ring.inv_pow2(1), ring.add(x0, x1)), x1
    if code == OP_I0Z1:
        return ring.mul(ring.inv_pow2(1), x0), x1
    return x0, x1


def simulate(sched, ring, x, seed=0):
    """Run the exported schedule on the cell list x (length L) in place."""
    rng = random.Random(seed)
    ordv = sched["ord"]
    jobs, progs, steps, ops = sched["jobs"], sched["progs"], sched["steps"], sched["ops"]
    for job_begin, job_count, _max_len in sched["passes"]:
        for base, stride, prog, s, nload, nstore in jobs[job_begin:job_begin + job_count]:
            step_begin, step_count, ln = progs[prog]
            loc = [x[base + i * stride] if i < nload else _rand(ring, rng) for i in range(ln)]
            for op_begin, op_count in steps[step_begin:step_begin + step_count]:
                # the base cases of one step run at the same time on the GPU
                # (one wave each): they must touch disjoint cells
                touched = set()
                for code, i0, i1, alog, b in ops[op_begin:op_begin + op_count]:
                    cells = {i0, i1}
                    assert not (cells & touched), "base cases of one step share a cell"
                    touched |= cells
                    e = (s * (1 << alog) + b) % ordv
                    loc[i0], loc[i1] = apply_op(ring, code, loc[i0], loc[i1], e)
            for i in range(nstore):
                x[base + i * stride] = loc[i]
    return x
