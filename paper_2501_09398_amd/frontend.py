"""Automatic iteration batching of a user step function: the automatic
conversion of an iterative GPU loop into iteration batches, with the batch
size chosen by the performance model, which the paper leaves to future work
(Sec. VI).

A *step* is any Python callable that enqueues GPU work on the current torch
stream and advances its state tensors by one iteration in place, so that
the same kernels on the same memory always advance the state by one more
iteration.  ``BatchedLoop(step).run(n, b)``:

* ``b = 0``: calls the step n times (one launch sequence per iteration, the
  baseline loop of Listings 1-2);
* ``b >= 1``: records b consecutive calls into one HIP graph by stream
  capture (``torch.cuda.CUDAGraph``; the capture builder of Sec. II),
  replays it floor(n/b) times and calls the step for the n mod b remaining
  iterations (loop peeling, Sec. VI).  Graphs are cached per b.

``tune(n)`` picks b with the paper's model: for each admissible b (the
divisors of n up to ``max_b``, Eq. 4) it times the capture (T_C, Eq. 2
fitted against b) and the replays of a probe of the loop (T_E, Eq. 6 fitted
against b and scaled to n iterations; both of Eq. 6's terms are linear in
the iteration count), and minimises Eq. 1.

Requirements on the step: replayable (no host synchronisation, no host-side
decisions on device values, no reallocation of the state).  A step that
alternates between buffers through Python state (it swaps references after
each call) is only replayable with a b that brings the references back to
where they were: a graph bakes in the buffers of the calls it recorded, so
after an odd b of a two-buffer step the second replay would read the wrong
buffer.  Give such a step's buffer list as ``state`` (the mutable list of
tensors that the step reorders): each capture compares it before and after
the b recorded calls and, if the buffers moved, puts the list back and
raises ValueError.  Capture records whatever the step enqueues;
avoid library calls that record memset nodes (some reductions do), whose
replays after the first can differ.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import perfmodel as pm


class BatchedLoop:
    def __init__(self, step, device=None, state=None):
        self.step = step
        self.state = state          # the step's buffer list, which it may reorder (or None)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._graphs = {}

    def _capture(self, b):
        """Record b calls of the step; returns (graph, T_C seconds).
        Raises ValueError when the declared state does not come back to the
        same buffers after the b calls (the graph would replay from the
        wrong ones); the list is then put back as it was (the recorded
        calls ran no kernel)."""
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        before = list(self.state) if self.state is not None else None
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(b):
                self.step()
        torch.cuda.synchronize(self.device)
        if before is not None and [t.data_ptr() for t in self.state] != [t.data_ptr() for t in before]:
            self.state[:] = before
            raise ValueError(f"the step's buffers move over {b} calls, so a graph of {b} calls cannot be "
                             f"replayed: choose a b after which they are back in place (e.g. an even b for "
                             f"two alternating buffers)")
        return g, time.perf_counter() - t0

    def graph(self, b):
        """The cached graph of b iterations and the T_C spent on it now (0
        when it was cached)."""
        if b in self._graphs:
            return self._graphs[b], 0.0
        g, tc = self._capture(b)
        self._graphs[b] = g
        return g, tc

    def drop(self, b=None):
        """Forget the graph of b iterations (all graphs if b is None)."""
        if b is None:
            self._graphs.clear()
        else:
            self._graphs.pop(b, None)

    def run(self, n, b=0):
        """Advance n iterations; returns {"t_create_s", "t_exec_s",
        "graph_launches", "peeled"} with T_E from events on the current
        stream around all launches."""
        if n < 0 or b < 0:
            raise ValueError("n and b must be >= 0")
        nb, peel = (n // b, n % b) if b > 0 and n >= b else (0, n)
        g, tc = self.graph(b) if nb else (None, 0.0)
        s = torch.cuda.current_stream(self.device)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(nb):
            g.replay()
        for _ in range(peel):
            self.step()
        e1.record(s)
        e1.synchronize()
        return {"t_create_s": tc, "t_exec_s": e0.elapsed_time(e1) * 1e-3, "graph_launches": nb, "peeled": peel}

    def tune(self, n, candidates=None, max_b=2000, probe_iters=None, reps=2):
        """Choose b for a run of n iterations (Eqs. 1, 2, 6).  The probes
        advance the state: each candidate runs probe_iters iterations (n
        by default) `reps` times.  Returns {"b", "b_measured",
        "b_closed_form", "model", "sweep"} with the sweep as (b, T_C, T_E
        scaled to n)."""
        cands = sorted(candidates) if candidates else pm.divisors(n, 1, max_b)
        probe = probe_iters or n
        cands = [c for c in cands if c <= probe] or [1]
        sweep = []
        for b in cands:
            tcs, tes = [], []
            for _ in range(reps):
                self.drop(b)
                r = self.run(probe, b)
                tcs.append(r["t_create_s"])
                tes.append(r["t_exec_s"] * n / probe)
            self.drop(b)
            sweep.append((b, float(np.median(tcs)), float(np.median(tes))))
        S = np.array([s[0] for s in sweep], float)
        model = pm.Model(pm.fit_creation(S, [s[1] for s in sweep]), pm.fit_execution(S, [s[2] for s in sweep]), K=1)
        b_model, _ = model.best(cands)
        total = {s[0]: s[1] + s[2] for s in sweep}
        return {"b": b_model, "b_measured": min(total, key=total.get), "b_closed_form": model.s_closed_form(),
                "model": model.as_dict(), "sweep": sweep}


def batch(step, device=None, state=None):
    """BatchedLoop of a step function (see the module documentation)."""
    return BatchedLoop(step, device, state)
