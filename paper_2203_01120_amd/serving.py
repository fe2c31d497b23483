"""Continuous batching of susceptibility requests over the chain-level C ABI.

A request asks for chi(q, omega) of one system along one field direction:
(system, q set, direction, flavour, steps, omega grid, eta).  The server
admits requests as device-resident chains while their vectors fit a
device-memory budget.  Pending requests of the same system, q set and
flavour with similar step counts are admitted together as the lanes of one
chain (tm_chain_begin_multi, up to `lanes` of them): each step then applies
L to all of them in one pass.  The server advances every admitted chain in
rounds (whole step periods, more of them per round for the faster systems;
the chains of one system on that system's stream, different systems on
different streams so that their kernels run concurrently), and finishes a
request -- coefficients, then chi on its frequencies (tm_chi) -- as soon as
its lane has run its steps.  All arithmetic happens in the library; this
module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import binding as tb


@dataclass
class Request:
    rid: int
    system: str
    iq: int
    direction: str
    flavour: str
    nsteps: int
    omega: np.ndarray
    eta: float
    arrival: float = 0.0          # seconds on the server's clock
    # filled by the server
    chi: Optional[np.ndarray] = None
    coeffs: Optional[dict] = None
    t_admit: float = float("nan")
    t_done: float = float("nan")


@dataclass
class _Active:
    reqs: List[Request]                   # one per lane
    chain: int
    flavour: str
    cap: int
    issued: int = 0
    nbytes: int = 0
    done: List[bool] = field(default_factory=list)


@dataclass
class SystemSlot:
    handle: int
    nelem: Dict[int, int]                 # q set -> complex elements of a BR vector
    stream: object = None                 # torch.cuda.Stream
    active: List[_Active] = field(default_factory=list)
    period_s: float = 0.0                 # measured seconds per step period (EMA)
    periods: int = 1                      # periods per round


def chain_bytes(nelem: int, flavour: str, nsteps: int, lanes: int = 1) -> int:
    """Device bytes of one chain: per lane its BR vectors (pH 5, nH 9) and
    coefficients, plus the 4 shared measure vectors."""
    nvec = lanes * (5 if flavour == "pH" else 9) + 4
    return nvec * nelem * 16 + lanes * nsteps * 104


class Server:
    """Admission by device-memory budget, round-robin stepping, per-system streams."""

    PERIOD = {"pH": 6, "nH": 3}

    def __init__(self, systems: Dict[str, SystemSlot], budget_bytes: int, rounds_per_sync: int = 1,
                 lanes: int = 4, lane_slack: float = 1.25, max_chains: int = 0, chain_slots: int = 1):
        import torch
        self.torch = torch
        self.systems = systems
        for s in systems.values():
            if s.stream is None:
                s.stream = torch.cuda.Stream()   # default priority
            # the systems already overlap on their own streams; chain_slots > 1
            # also overlaps the chains of one system (library streams)
            tb.tm_system_set_chain_slots(s.handle, chain_slots)
        self.budget = int(budget_bytes)
        self.used = 0
        self.pending: deque = deque()
        self.done: List[Request] = []
        self.rounds_per_sync = rounds_per_sync
        self.lanes = max(1, min(4, int(lanes)))
        self.lane_slack = lane_slack         # longest / shortest request of one chain, at most
        # chains per system at a time (0: no limit); requests beyond it wait and
        # are admitted together as the lanes of a later chain
        self.max_chains = int(max_chains)
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> None:
        self.pending.append(req)

    def idle(self) -> bool:
        return not self.pending and all(not s.active for s in self.systems.values())

    def _bytes(self, group: List[Request]) -> int:
        head = group[0]
        return chain_bytes(self.systems[head.system].nelem[head.iq], head.flavour, max(r.nsteps for r in group),
                           len(group))

    def _group(self, head: Request) -> List[Request]:
        """The head request and up to lanes-1 pending partners for one chain
        (same system, q set and flavour, similar step counts, within the budget)."""
        group = [head]
        for r in self.pending:
            if len(group) == self.lanes:
                break
            if (r.system, r.iq, r.flavour) != (head.system, head.iq, head.flavour):
                continue
            steps = [q.nsteps for q in group] + [r.nsteps]
            if max(steps) > self.lane_slack * min(steps):
                continue
            if self.used + self._bytes(group + [r]) > self.budget:
                continue
            group.append(r)
        return group

    def _admit(self) -> None:
        """FIFO over the pending requests, skipping systems at their chain limit;
        stops at the first chain that does not fit the memory budget."""
        i = 0
        while i < len(self.pending):
            head = self.pending[i]
            slot = self.systems[head.system]
            if self.max_chains and len(slot.active) >= self.max_chains:
                i += 1
                continue
            del self.pending[i]
            group = self._group(head)
            cap = max(r.nsteps for r in group)
            nb = self._bytes(group)
            if self.used + nb > self.budget and self.used > 0:
                self.pending.insert(i, head)
                return
            for r in group[1:]:
                self.pending.remove(r)
            h = tb.tm_chain_begin_multi(slot.handle, head.iq, [r.direction for r in group], head.flavour, cap,
                                        stream=slot.stream.cuda_stream)
            now = self.now()
            for r in group:
                r.t_admit = now
            slot.active.append(_Active(group, h, head.flavour, cap, 0, nb, [False] * len(group)))
            self.used += nb

    def _finish_lanes(self, a: _Active) -> None:
        """Finishes every request whose lane has run its steps."""
        lanes = None
        for i, r in enumerate(a.reqs):
            if a.done[i] or a.issued < r.nsteps:
                continue
            if lanes is None:
                lanes = tb.tm_chain_coeffs_lanes(a.chain, a.cap)
            co = lanes[i]
            n = r.nsteps
            mine = {k: co[k][..., :n].copy() for k in ("alpha", "beta", "gamma", "z", "zn")}
            mine.update(n1=co["n1"], steps_done=min(co["steps_done"], n), breakdown=co["steps_done"] < n)
            r.coeffs = mine
            r.chi = tb.tm_chi(mine, max(1, mine["steps_done"]), r.omega, r.eta)
            r.t_done = self.now()
            a.done[i] = True
            self.done.append(r)

    def round(self) -> None:
        """Admit what fits, advance the active chains, finish completed ones.

        A round gives each system enough step periods that all systems take
        about as long as one period of the slowest one, so fast systems do not
        idle behind slow ones at the round's synchronisation."""
        torch = self.torch
        self._admit()
        busy = [s for s in self.systems.values() if s.active]
        slow = max((s.period_s for s in busy), default=0.0)
        marks = []
        for slot in busy:
            if slot.period_s > 0 and slow > 0:
                slot.periods = int(max(1, min(64, round(slow / slot.period_s))))
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(slot.stream)
            for flav in ("pH", "nH"):
                group = [a for a in slot.active if a.flavour == flav]
                if not group:
                    continue
                k = self.PERIOD[flav] * slot.periods * self.rounds_per_sync
                tb.tm_chains_step([a.chain for a in group], k, stream=slot.stream.cuda_stream)
                for a in group:
                    a.issued = min(a.cap, a.issued + k)
            ev1.record(slot.stream)
            marks.append((slot, ev0, ev1))
        for slot, ev0, ev1 in marks:
            ev1.synchronize()
            per = ev0.elapsed_time(ev1) * 1e-3 / (slot.periods * self.rounds_per_sync)
            slot.period_s = per if slot.period_s == 0 else 0.7 * slot.period_s + 0.3 * per
        for slot in self.systems.values():
            keep = []
            for a in slot.active:
                self._finish_lanes(a)
                if all(a.done):
                    tb.tm_chain_end(a.chain)
                    self.used -= a.nbytes
                else:
                    keep.append(a)
            slot.active = keep

    def run(self, requests: List[Request]) -> List[Request]:
        """Replay requests at their arrival times (seconds from now); returns them completed."""
        todo = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        i = 0
        while i < len(todo) or not self.idle():
            t = self.now()
            while i < len(todo) and todo[i].arrival <= t:
                self.submit(todo[i])
                i += 1
            if self.idle():
                if i < len(todo):
                    time.sleep(max(0.0, todo[i].arrival - self.now()))
                continue
            self.round()
        return self.done


def run_one_at_a_time(systems: Dict[str, SystemSlot], requests: List[Request]) -> List[Request]:
    """Reference path: FIFO, one request at a time, every kernel issued directly (no graphs)."""
    import torch
    tb.tm_chains_use_graphs(False)
    try:
        t0 = time.perf_counter()
        for req in sorted(requests, key=lambda r: r.arrival):
            now = time.perf_counter() - t0
            if req.arrival > now:
                time.sleep(req.arrival - now)
            req.t_admit = time.perf_counter() - t0
            co = tb.tm_lanczos_run(systems[req.system].handle, req.iq, req.direction, req.flavour, req.nsteps)
            m = max(1, min(co["steps_done"], req.nsteps))
            req.coeffs = co
            req.chi = tb.tm_chi(co, m, req.omega, req.eta)
            torch.cuda.synchronize()
            req.t_done = time.perf_counter() - t0
    finally:
        tb.tm_chains_use_graphs(True)
    return requests


def summary(reqs: List[Request]) -> dict:
    lat = np.array([r.t_done - r.arrival for r in reqs])
    span = max(r.t_done for r in reqs) - min(r.arrival for r in reqs)
    return {"spectra_per_s": round(len(reqs) / span, 4), "p50_s": round(float(np.percentile(lat, 50)), 4),
            "p99_s": round(float(np.percentile(lat, 99)), 4), "requests": len(reqs),
            "steps": int(sum(r.coeffs["steps_done"] for r in reqs)),
            "breakdowns": int(sum(bool(r.coeffs["breakdown"]) for r in reqs))}
