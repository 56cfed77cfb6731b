"""Batches in flight: the factorisation of later batches runs while batch k
is solved.

Both phases of one batch are latency-bound chains of small launches (one
launch per panel step of the block factorisation, one per block row of a
sweep), and neither fills the GPU: a factor step keeps about two
workgroups per compute unit busy, a sweep step four.  Independent batches
(the frequencies of different models, or successive requests) can therefore
share the GPU: batch k+1 (and with factor_streams = f > 1, batches up to
k+f, side by side) is factored while batch k is solved on another stream,
each stream driven by its own host thread (the library holds no
global lock, and ctypes releases the interpreter lock for the duration of
a call).  Every batch is still factored and solved completely,
with the same kernels and arithmetic as the serial schedule, so the results
are bitwise those of solve_batch(factor_batch(...)).

    pipe = Pipeline(factor_streams=1)
    results = pipe.run(batches)   # [(X list, info list)] per batch
"""
from __future__ import annotations

import dataclasses
import threading

from . import helm


@dataclasses.dataclass
class Batch:
    grids: list
    ms: list
    omegas: list
    Bs: list                     # per system, [S][N] complex128 device tensors
    precision: str = "fp32_ir"
    tol: float = 1e-10
    out: list = None             # optional output tensors, one per system


class Pipeline:
    """factor_streams factorisations run side by side (each on its own
    stream and host thread; batch k goes to worker k mod factor_streams)
    while the batches already factored are solved in order on one more
    stream.  At most factor_streams + 1 batches hold factors at a time: a
    worker starts batch k once batch k - factor_streams - 1 is solved."""

    def __init__(self, factor_streams: int = 1):
        if factor_streams < 1:
            raise ValueError("factor_streams must be >= 1")
        self.nf = int(factor_streams)
        # the process's pipeline streams (helm.pooled_stream): a second
        # Pipeline with new streams ran with no overlap at all (its factor and
        # solve streams shared a hardware queue)
        self.s_factor = [helm.pooled_stream(("pipeline factor", j)) for j in range(self.nf)]
        self.s_solve = helm.pooled_stream("pipeline solve")

    # Each call runs with its own stream current: the inputs were made ready
    # when run() started, so the binding has nothing to order it after (a
    # wait on the caller's stream from every call cost up to 5% here).
    def _factor(self, b: Batch, j: int):
        torch = helm._torch()
        with torch.cuda.stream(self.s_factor[j]):
            return helm.factor_batch(b.grids, b.ms, b.omegas, b.precision, stream=self.s_factor[j])

    def _solve(self, b: Batch, Fs):
        torch = helm._torch()
        with torch.cuda.stream(self.s_solve):
            return helm.solve_batch(Fs, b.Bs, tol=b.tol, stream=self.s_solve, out=b.out)

    def run(self, batches):
        """Factor and solve every batch; returns [(Xs, infos)] in order."""
        torch = helm._torch()
        torch.cuda.current_stream().synchronize()   # inputs written on the caller's stream
        n = len(batches)
        results = [None] * n
        if not n:
            return results
        facs = [None] * n
        ready = [threading.Event() for _ in range(n)]
        solved = [threading.Event() for _ in range(n)]
        stop = threading.Event()
        err = []

        def worker(j):
            for k in range(j, n, self.nf):
                if k - self.nf - 1 >= 0:
                    solved[k - self.nf - 1].wait()
                if stop.is_set():
                    ready[k].set()
                    continue
                try:
                    facs[k] = self._factor(batches[k], j)
                except BaseException as e:   # re-raised on the calling thread
                    err.append(e)
                    stop.set()
                ready[k].set()

        threads = [threading.Thread(target=worker, args=(j,)) for j in range(self.nf)]
        for t in threads:
            t.start()
        try:
            for k in range(n):
                ready[k].wait()
                if err or facs[k] is None:
                    break
                results[k] = self._solve(batches[k], facs[k])
                self.s_solve.synchronize()
                for F in facs[k]:
                    F.close()
                facs[k] = None
                solved[k].set()
        except BaseException as e:
            err.append(e)
        finally:
            stop.set()
            for ev in solved:
                ev.set()
            for t in threads:
                t.join()
            for Fs in facs:
                for F in Fs or []:
                    F.close()
        if err:
            raise err[0]
        return results
