"""Spill-policy simulators for run generation with early aggregation:
read-sort-write cycles (``simulate``) and replacement selection through the
index (``simulate_replacement``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Run generation absorbs input into an ordered in-memory index of unique keys;
a key already in the index is absorbed, a new key is inserted; when memory is
full the whole index is written, in key order, as one run and emptied
(read-sort-write cycles, the policy the paper's product implementation uses:
Section 3 on run generation with an in-memory index, Section 6.1 on the
product implementation).  The final index is not written out; it joins the
final merge as one more input (the paper's analysis likewise ignores the
in-memory run, Section 3, Example 2).

Batch-granular reading of "memory is full": input is consumed in batches of
``batch_rows`` consecutive rows.  A batch's distinct keys are absorbed into the
index if the union fits ``capacity`` keys; otherwise the index is spilled as a
run and the batch's distinct keys start the next index.  The simulator works on
key sets only, so it yields the exact run count and spilled-row count for that
policy, independently of how a batch is sorted.
"""
from __future__ import annotations

import numpy as np


def simulate(keys, batch_rows: int, capacity: int, keep_runs: bool = False, absorb_first: bool = False):
    """Read-sort-write cycles at batch granularity (see the module docstring).
    With ``keep_runs`` the result also holds ``run_keys``: each run's sorted
    keys, in the order the runs were written.

    ``absorb_first`` is the other batch-granular reading of "memory is full":
    every batch is absorbed, and as soon as the index then holds more than
    ``capacity`` keys it is written whole as one run (up to capacity plus a
    batch) and the next index starts empty; the memory holds up to capacity
    plus one batch of keys.  This is the rule of an index that absorbs a batch
    in place, where the index before the absorb no longer exists."""
    if batch_rows <= 0 or capacity <= 0 or batch_rows > capacity:
        raise ValueError("need 0 < batch_rows <= capacity")
    keys = np.asarray(keys, dtype=np.uint64)
    index = np.empty(0, np.uint64)
    run_sizes = []
    run_keys = []
    for start in range(0, keys.shape[0], batch_rows):
        batch = np.unique(keys[start:start + batch_rows])
        merged = np.union1d(index, batch)
        if merged.shape[0] <= capacity:
            index = merged
        elif absorb_first:
            run_sizes.append(int(merged.shape[0]))
            if keep_runs:
                run_keys.append(merged)
            index = np.empty(0, np.uint64)
        else:
            run_sizes.append(int(index.shape[0]))
            if keep_runs:
                run_keys.append(index)
            index = batch
    out = {"runs": len(run_sizes), "spilled_rows": int(sum(run_sizes)),
           "run_sizes": run_sizes, "final_index_rows": int(index.shape[0])}
    if keep_runs:
        out["run_keys"] = run_keys
    return out


def simulate_hybrid(keys, batch_rows: int, resident_capacity: int, run_capacity: int):
    """Hybrid run generation (Section 5, hybrid algorithms): part of memory
    holds an in-memory index that removes duplicates of the key values
    assigned to it, for good; the rest generates runs for the other key
    values by read-sort-write cycles.

    Batch-granular reading, with the assignment of key values made as the
    input arrives: the resident index holds every key below a cut, which
    starts above every key.  A batch's distinct keys below the cut join the
    resident index; when it then holds more than ``resident_capacity`` keys,
    its largest keys beyond the smallest three quarters of that capacity are
    written, in key order, as one run and the cut moves down to the smallest
    of them (those key values are from then on assigned to runs).  The batch's
    keys at or above the cut are absorbed into the run-generation index if
    the union fits ``run_capacity`` keys; otherwise that index is written as
    a run and those keys start the next one.  A batch's keys at or above the
    cut are split off before the demotion that the batch may cause.  Both
    indexes stay in memory at the end.  Runs are listed in the order they are
    written (per batch: the run-generation index first, then a demotion)."""
    if batch_rows <= 0 or batch_rows > run_capacity or (0 < resident_capacity < 4) or resident_capacity < 0:
        raise ValueError("need 0 < batch_rows <= run_capacity and resident_capacity 0 or >= 4")
    keys = np.asarray(keys, dtype=np.uint64)
    keep = resident_capacity * 3 // 4
    resident = np.empty(0, np.uint64)
    gen = np.empty(0, np.uint64)
    # a Python int: every key is below it; with no resident index every key
    # is assigned to runs from the start
    cut = 1 << 64 if resident_capacity else 0
    run_sizes = []
    kinds = []
    for start in range(0, keys.shape[0], batch_rows):
        batch = np.unique(keys[start:start + batch_rows])
        if cut >= 1 << 64:
            p = batch.shape[0]
        else:
            p = int(np.searchsorted(batch, np.uint64(cut), "left"))
        lo, hi = batch[:p], batch[p:]
        # run generation for the keys assigned to runs
        merged = np.union1d(gen, hi)
        if merged.shape[0] <= run_capacity:
            gen = merged
        else:
            run_sizes.append(int(gen.shape[0]))
            kinds.append("run")
            gen = hi
        # the resident index
        resident = np.union1d(resident, lo)
        if resident.shape[0] > resident_capacity:
            demoted = resident[keep:]
            run_sizes.append(int(demoted.shape[0]))
            kinds.append("demotion")
            cut = int(demoted[0])
            resident = resident[:keep]
    return {"runs": len(run_sizes), "spilled_rows": int(sum(run_sizes)), "run_sizes": run_sizes,
            "run_kinds": kinds, "final_index_rows": int(resident.shape[0] + gen.shape[0]),
            "resident_rows": int(resident.shape[0]), "cut": cut}


def model_spill_rows(I: float, M: float, O: float) -> float:
    """Predicted total size of the initial runs with an in-memory index and
    memory kept full (Section 3, Example 2): zero when the output fits memory,
    otherwise M + (1 - M/O) * I.  An approximation (it assumes replacement
    selection and uniformly distributed keys)."""
    if O <= M:
        return 0.0
    return M + (1.0 - M / O) * I


def simulate_replacement(keys, batch_rows: int, capacity: int):
    """Run generation by replacement selection through the in-memory index
    (Section 3: the index supports replacement selection as well as
    read-sort-write cycles; eviction scans the index in key order, so runs grow
    to about twice the memory for random input with no extra comparison and no
    run flag per row).

    Batch-granular reading: a batch's distinct keys join the index.  If the
    union holds e > capacity keys more than capacity, the e smallest keys at or
    after the scan cursor are evicted in key order and appended to the open
    run, and the cursor moves just past the last evicted key.  When the scan
    passes the largest key before e keys are evicted, the open run ends and
    the scan restarts at the smallest key with a new run.  Keys below the
    cursor (inserted after the scan passed them) wait for the next run.  The
    final index is not written out."""
    if batch_rows <= 0 or capacity <= 0 or batch_rows > capacity:
        raise ValueError("need 0 < batch_rows <= capacity")
    keys = np.asarray(keys, dtype=np.uint64)
    index = np.empty(0, np.uint64)
    cursor = 0            # a Python int; 2**64 once the scan passed the largest key value
    open_rows = 0
    run_sizes = []
    for start in range(0, keys.shape[0], batch_rows):
        merged = np.union1d(index, np.unique(keys[start:start + batch_rows]))
        m = merged.shape[0]
        if m <= capacity:
            index = merged
            continue
        e = m - capacity
        p = m if cursor >= 1 << 64 else int(np.searchsorted(merged, np.uint64(cursor), "left"))
        a = min(e, m - p)
        keep = np.ones(m, bool)
        keep[p:p + a] = False
        open_rows += a
        last = int(merged[p + a - 1]) if a else None
        if a < e:
            # the scan passed the largest key: the open run ends
            if open_rows:
                run_sizes.append(open_rows)
            b = e - a
            keep[:b] = False
            open_rows = b
            last = int(merged[b - 1])
        cursor = last + 1
        index = merged[keep]
    if open_rows:
        run_sizes.append(open_rows)
    return {"runs": len(run_sizes), "spilled_rows": int(sum(run_sizes)),
            "run_sizes": run_sizes, "final_index_rows": int(index.shape[0])}


def preliminary_merges(run_rows, fan_in: int, out_bound: float):
    """Traditional merge steps that bring the run count down to the fan-in of
    a final merge (Section 4, Example 4 and its note on the merge steps;
    Section 4.4: such steps precede a wide merge that cannot absorb all runs).

    Each step merges the smallest runs.  The first step takes just enough runs
    that every later step can merge a full fan-in and the last one leaves
    exactly ``fan_in`` runs: with n runs it merges (n - fan_in) mod
    (fan_in - 1) + 1 of them when that remainder is nonzero.  Aggregation
    within a merge bounds a step's output by the final output size
    ``out_bound``.  Returns the run count after each step and the rows the
    steps write (their spill volume beyond the initial runs)."""
    runs = sorted(float(r) for r in run_rows)
    counts = [len(runs)]
    written = 0.0
    F = int(fan_in)
    if F < 2:
        raise ValueError("fan-in below 2")
    first = True
    while len(runs) > F:
        extra = (len(runs) - F) % (F - 1)
        take = extra + 1 if first and extra else F
        first = False
        merged = min(sum(runs[:take]), float(out_bound))
        runs = sorted(runs[take:] + [merged])
        written += merged
        counts.append(len(runs))
    return {"counts": counts, "written_rows": written, "final_runs": runs}


def preliminary_merges_exact(run_keys, fan_in: int):
    """The same merge steps on actual runs (their sorted key sets): a step
    takes the smallest runs, ties broken by the order in which runs were
    written (a merged run counts as written when its step ends), and writes
    the union of their keys as one run, since equal keys combine.  Returns the
    run count after each step, the rows each step wrote, their total, and the
    final runs' sizes in written order."""
    F = int(fan_in)
    if F < 2:
        raise ValueError("fan-in below 2")
    runs = [(np.asarray(r, dtype=np.uint64), i) for i, r in enumerate(run_keys)]
    seq = len(runs)
    counts = [len(runs)]
    step_rows = []
    first = True
    while len(runs) > F:
        extra = (len(runs) - F) % (F - 1)
        take = extra + 1 if first and extra else F
        first = False
        order = sorted(range(len(runs)), key=lambda j: (runs[j][0].shape[0], runs[j][1]))
        chosen = set(order[:take])
        merged = np.unique(np.concatenate([runs[j][0] for j in order[:take]]))
        runs = [r for j, r in enumerate(runs) if j not in chosen] + [(merged, seq)]
        seq += 1
        step_rows.append(int(merged.shape[0]))
        counts.append(len(runs))
    return {"counts": counts, "step_rows": step_rows, "written_rows": int(sum(step_rows)),
            "final_run_sizes": [int(r[0].shape[0]) for r in runs]}


def hybrid_plan(I: float, M: float, O: float, F: int, P: float = None):
    """Hybrid run generation (Section 5, hybrid algorithms): the smallest
    fan-out f with O <= f*M + (1 - f/F)*M, i.e. f = ceil((O - M)/(M - P)),
    gives the memory fraction f/F to run generation and the rest to an
    in-memory index that absorbs (1 - f/F)*M of the output, i.e. that share
    of the input.  Runs of read-sort-write cycles hold f/F*M rows.  Returns
    f, the output fraction the index absorbs, the spilled rows, the run
    count, and whether one wide merge suffices (O <= F*M).  P defaults to
    M/F (pages per memory load equal to the fan-in)."""
    import math
    if P is None:
        P = M / F
    f = max(0, math.ceil((O - M) / (M - P))) if O > M else 0
    f = min(f, F)
    index_out = (1.0 - f / F) * M
    absorbed = min(1.0, index_out / O)
    spilled = (1.0 - absorbed) * I
    run_rows = f / F * M
    runs = spilled / run_rows if run_rows else 0.0
    return {"f": f, "index_output_fraction": absorbed, "spilled_rows": spilled, "run_rows": run_rows,
            "runs": runs, "single_wide_merge": O <= F * M}


def traditional_levels(n_runs: int, F: int):
    """Level-wise traditional merging of n equal runs with fan-in F: merge
    levels and merge steps until one run remains (Section 5's hybrid example:
    1,000 runs at fan-in 10 take three levels and 111 steps)."""
    levels = steps = 0
    n = int(n_runs)
    while n > 1:
        m = -(-n // F)
        steps += m
        n = m
        levels += 1
    return levels, steps
