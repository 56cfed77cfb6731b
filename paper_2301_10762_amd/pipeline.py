"""Two batches in flight: the factorisation of batch k+1 runs while batch k
is solved.

Both phases of one batch are latency-bound chains of small launches (one
launch per panel step of the block factorisation, one per block row of a
sweep), and neither fills the GPU: a factor step keeps about two
workgroups per compute unit busy, a sweep step four.  Independent batches
(the frequencies of different models, or successive requests) can therefore
share the GPU: batch k+1 is factored on one stream while batch k is solved
on another, each driven by its own host thread (the library holds no
global lock, and ctypes releases the interpreter lock for the duration of
a call).  Every batch is still factored and solved completely,
with the same kernels and arithmetic as the serial schedule, so the results
are bitwise those of solve_batch(factor_batch(...)).

    pipe = Pipeline()
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
    def __init__(self):
        torch = helm._torch()
        self.s_factor = torch.cuda.Stream()
        self.s_solve = torch.cuda.Stream()

    def _factor(self, b: Batch):
        return helm.factor_batch(b.grids, b.ms, b.omegas, b.precision, stream=self.s_factor)

    def _solve(self, b: Batch, Fs):
        return helm.solve_batch(Fs, b.Bs, tol=b.tol, stream=self.s_solve, out=b.out)

    def run(self, batches):
        """Factor and solve every batch; returns [(Xs, infos)] in order."""
        torch = helm._torch()
        torch.cuda.current_stream().synchronize()   # inputs written on the caller's stream
        results = [None] * len(batches)
        if not batches:
            return results
        Fs = self._factor(batches[0])
        for k in range(len(batches)):
            nxt, err = {}, []

            def factor_next():
                try:
                    if k + 1 < len(batches):
                        nxt["F"] = self._factor(batches[k + 1])
                except BaseException as e:   # re-raised on the calling thread
                    err.append(e)

            def solve_this():
                try:
                    results[k] = self._solve(batches[k], Fs)
                except BaseException as e:
                    err.append(e)

            ta = threading.Thread(target=factor_next)
            ta.start()
            solve_this()
            ta.join()
            self.s_solve.synchronize()
            for F in Fs:
                F.close()
            if err:
                for F in nxt.get("F", []):
                    F.close()
                raise err[0]
            Fs = nxt.get("F")
        return results
