"""Continuous batching of susceptibility requests over the chain-level C ABI.

A request asks for chi(q, omega) of one system along one field direction:
(system, q set, direction, flavour, steps, omega grid, eta).  The server
admits requests as device-resident chains while everything they need fits a
device-memory budget, and it counts all of it:

* every loaded system's footprint -- its tables (ground-state bands,
  occupied partners, projectors, fields), its ground state in the form the
  plane kernels read (the resident real-space copy, capped per system, or
  the z-transformed columns) and its apply workspaces (one per chain slot,
  as wide as the widest chain) -- from tm_system_footprint before the
  system exists and tm_system_memory once it does;
* every chain's vectors and coefficients.

Systems come in two kinds: ones the caller created (kept for the server's
life) and specs that the server creates when a request needs them and
destroys, least recently used first, when another system needs the memory
and they have no chain running.

Pending requests of the same system and flavour with similar step counts
are admitted together as the lanes of one chain (tm_chain_begin_lanes, up to
`lanes` of them; requests on different q sets of a system share a chain once
the system holds its ground state resident in real space, which lanes of
different q sets need): each step then applies L to all of them in one pass.  The server advances every admitted chain in rounds
(whole step periods, more of them per round for the faster systems; the
chains of one system on that system's stream, different systems on different
streams so that their kernels run concurrently), and finishes a request --
coefficients, then chi on its frequencies (tm_chi) -- as soon as its lane
has run its steps.  A chain that breaks down before its first step (the
start vector has no weight in the metric, e.g. the Goldstone direction at
q = 0) finishes with chi = 0 and `breakdown` set.  All arithmetic happens in
the library; this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

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
    error: Optional[str] = None
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
class SystemSpec:
    """A system the server creates on demand: `make_desc` builds its
    descriptor (host work; called once, the result is kept);
    `resident_cap` bounds its resident real-space ground state in bytes
    (-1: the whole copy; 0: always the column path)."""
    make_desc: Callable[[], "tb.SystemDesc"]
    resident_cap: int = -1


@dataclass
class SystemSlot:
    handle: int
    nelem: Dict[int, int]                 # q set -> complex elements of a BR vector
    stream: object = None                 # torch.cuda.Stream
    active: List[_Active] = field(default_factory=list)
    period_s: float = 0.0                 # measured seconds per step period (EMA)
    periods: int = 1                      # periods per round
    footprint: int = 0                    # device bytes charged to the budget
    spec: Optional[str] = None            # created from this spec (evictable) or None (the caller's)
    last_used: float = 0.0


def chain_bytes(nelem: int, flavour: str, nsteps: int, lanes: int = 1, mixed: bool = False) -> int:
    """Device bytes of one chain: per lane its BR vectors (pH 5, nH 9) and
    coefficients, plus the 4 measure vectors (one set per lane when the lanes
    carry different q sets)."""
    nvec = lanes * (5 if flavour == "pH" else 9) + 4 * (lanes if mixed else 1)
    return nvec * nelem * 16 + lanes * nsteps * 104


def _plan(mem: dict, budget: int, resident_cap: int, lanes: int, slots: int):
    """(footprint bytes, resident limit) of a system from its memory figures:
    the resident copy when it is within the cap and the budget (its column
    cache is built on the way, so both are counted), else the columns."""
    ws = mem["workspace_per_rhs"] * lanes * slots
    cap = mem["resident_full"] if resident_cap < 0 else resident_cap
    full = mem["resident_full"]
    if 0 < full <= cap and mem["tables"] + full + mem["columns_full"] + ws <= budget:
        return mem["tables"] + full + mem["columns_full"] + ws, full
    return mem["tables"] + mem["columns_full"] + ws, 0


class SystemPool:
    """Loaded systems under a device-memory budget: the caller's systems
    (pinned) and systems created from specs on demand, evicted least recently
    used first when idle."""

    def __init__(self, systems: Dict[str, SystemSlot], budget_bytes: int, specs: Optional[Dict[str, SystemSpec]] = None,
                 lanes: int = 1, chain_slots: int = 1):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.specs = dict(specs or {})
        self.lanes = lanes
        self.chain_slots = chain_slots
        self.systems: Dict[str, SystemSlot] = {}
        self.used = 0
        self._descs: Dict[str, object] = {}
        self._mem: Dict[str, dict] = {}
        self.created = 0
        self.evicted = 0
        for name, slot in systems.items():
            self._register(name, slot, -1)

    def _register(self, name: str, slot: SystemSlot, resident_cap: int) -> None:
        torch = self.torch
        if slot.stream is None:
            slot.stream = torch.cuda.Stream()   # default priority
        tb.tm_system_set_chain_slots(slot.handle, self.chain_slots)
        mem = tb.tm_system_memory(slot.handle)
        foot, limit = _plan(mem, self.budget, resident_cap, self.lanes, self.chain_slots)
        tb.tm_system_set_resident_limit(slot.handle, limit)
        slot.footprint = foot
        slot.last_used = time.perf_counter()
        self.systems[name] = slot
        self.used += foot

    def desc(self, name: str):
        if name not in self._descs:
            self._descs[name] = self.specs[name].make_desc()
        return self._descs[name]

    def footprint(self, name: str) -> int:
        """Device bytes the system holds, or will hold once created."""
        if name in self.systems:
            return self.systems[name].footprint
        if name not in self._mem:
            self._mem[name] = tb.tm_system_footprint(self.desc(name))
        return _plan(self._mem[name], self.budget, self.specs[name].resident_cap, self.lanes, self.chain_slots)[0]

    def idle(self, name: str) -> bool:
        return not self.systems[name].active

    def acquire(self, name: str, extra: int) -> Optional[SystemSlot]:
        """The loaded system `name`, created if needed, with `extra` more bytes
        charged; None when they do not fit even after evicting every idle
        spec-created system."""
        need = extra + (0 if name in self.systems else self.footprint(name))
        if self.used + need > self.budget:
            idle = sorted((s.last_used, n) for n, s in self.systems.items()
                          if n != name and s.spec is not None and not s.active)
            for _, n in idle:
                if self.used + need <= self.budget:
                    break
                self.evict(n)
        if self.used + need > self.budget:
            return None
        if name not in self.systems:
            d = self.desc(name)
            h = tb.tm_system_create(d)
            nelem = {iq: tb.tm_qset_info_get(h, iq)["nelem"] for iq in range(np.atleast_2d(d.xq).shape[0])}
            slot = SystemSlot(handle=h, nelem=nelem, spec=name)
            try:
                self._register(name, slot, self.specs[name].resident_cap)
            except Exception:
                tb.tm_system_destroy(h)
                raise
            self.created += 1
        slot = self.systems[name]
        self.used += extra
        slot.last_used = time.perf_counter()
        return slot

    def release(self, nbytes: int) -> None:
        self.used -= nbytes

    def evict(self, name: str) -> None:
        slot = self.systems[name]
        assert slot.spec is not None and not slot.active
        self.torch.cuda.synchronize()
        tb.tm_system_destroy(slot.handle)
        self.used -= slot.footprint
        del self.systems[name]
        self.evicted += 1

    def close(self) -> None:
        """Destroys the systems created from specs (the caller's stay)."""
        for n in [n for n, s in self.systems.items() if s.spec is not None]:
            self.evict(n)


def _finish(r: Request, co: dict) -> None:
    """Coefficients of one request's lane (its first nsteps steps) and chi."""
    n = r.nsteps
    mine = {k: co[k][..., :n].copy() for k in ("alpha", "beta", "gamma", "z", "zn") if co.get(k) is not None}
    done = min(co["steps_done"], n)
    mine.update(n1=co["n1"], steps_done=done, breakdown=bool(co["breakdown"]) or co["steps_done"] < n)
    r.coeffs = mine
    if done == 0:
        # broke down at the start: no tridiagonal matrix, no spectrum
        r.chi = np.zeros((3, len(r.omega)), dtype=np.complex128)
        r.error = "breakdown before the first step"
    else:
        r.chi = tb.tm_chi(mine, done, r.omega, r.eta)


class Server:
    """Admission by device-memory footprint, round-robin stepping, per-system streams."""

    PERIOD = {"pH": 6, "nH": 3}

    def __init__(self, systems: Dict[str, SystemSlot], budget_bytes: int, rounds_per_sync: int = 1,
                 lanes: int = 4, lane_slack: float = 1.25, max_chains: int = 0, chain_slots: int = 1,
                 specs: Optional[Dict[str, SystemSpec]] = None):
        import torch
        self.torch = torch
        self.lanes = max(1, min(4, int(lanes)))
        # the systems already overlap on their own streams; chain_slots > 1
        # also overlaps the chains of one system (library streams)
        self.pool = SystemPool(systems, budget_bytes, specs, lanes=self.lanes, chain_slots=chain_slots)
        self.pending: deque = deque()
        self.done: List[Request] = []
        self.rounds_per_sync = rounds_per_sync
        self.lane_slack = lane_slack         # longest / shortest request of one chain, at most
        # chains per system at a time (0: no limit); requests beyond it wait and
        # are admitted together as the lanes of a later chain
        self.max_chains = int(max_chains)
        self.t0 = time.perf_counter()

    @property
    def systems(self) -> Dict[str, SystemSlot]:
        return self.pool.systems

    @property
    def used(self) -> int:
        return self.pool.used

    @property
    def budget(self) -> int:
        return self.pool.budget

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> None:
        if req.system not in self.pool.systems and req.system not in self.pool.specs:
            raise KeyError(f"unknown system {req.system}")
        self.pending.append(req)

    def idle(self) -> bool:
        return not self.pending and all(not s.active for s in self.systems.values())

    def _nelem(self, req: Request) -> int:
        if req.system in self.systems:
            return self.systems[req.system].nelem[req.iq]
        d = self.pool.desc(req.system)
        return _nelem_of_desc(d, req.iq)

    def _bytes(self, group: List[Request]) -> int:
        head = group[0]
        return chain_bytes(self._nelem(head), head.flavour, max(r.nsteps for r in group), len(group),
                           any(r.iq != head.iq for r in group))

    def _mixable(self, system: str) -> bool:
        """Whether lanes of different q sets may share a chain of this system:
        its ground state is resident in real space (decided at its first apply)."""
        slot = self.systems.get(system)
        return slot is not None and tb.tm_system_resident_bytes(slot.handle) > 0

    def _group(self, head: Request, room: int) -> List[Request]:
        """The head request and up to lanes-1 pending partners for one chain
        (same system and flavour -- and q set unless the system is resident --,
        similar step counts, within `room` bytes)."""
        group = [head]
        mix = self._mixable(head.system)
        for r in self.pending:
            if len(group) == self.lanes:
                break
            if (r.system, r.flavour) != (head.system, head.flavour) or (r.iq != head.iq and not mix):
                continue
            steps = [q.nsteps for q in group] + [r.nsteps]
            if max(steps) > self.lane_slack * min(steps):
                continue
            if self._bytes(group + [r]) > room:
                continue
            group.append(r)
        return group

    def _admit(self) -> None:
        """FIFO over the pending requests, skipping systems at their chain limit;
        stops at the first request whose chain (and system) does not fit."""
        i = 0
        while i < len(self.pending):
            head = self.pending[i]
            slot = self.systems.get(head.system)
            if slot is not None and self.max_chains and len(slot.active) >= self.max_chains:
                i += 1
                continue
            try:
                sysb = 0 if slot is not None else self.pool.footprint(head.system)
            except tb.TmError as e:
                # the library refuses the system (e.g. an unsupported grid): fail
                # its request rather than the server
                del self.pending[i]
                self._fail(head, f"system cannot be created: {e}")
                continue
            if sysb + self._bytes([head]) > self.budget:
                # can never fit: fail it rather than block the queue
                del self.pending[i]
                self._fail(head, "does not fit the device-memory budget")
                continue
            del self.pending[i]
            group = self._group(head, self.budget - self.used - sysb)
            nb = self._bytes(group)
            try:
                slot = self.pool.acquire(head.system, nb)
            except tb.TmError as e:
                # creation failed (nothing was charged): this request fails, its
                # would-be partners stay pending
                self._fail(head, f"system cannot be created: {e}")
                continue
            if slot is None:
                self.pending.insert(i, head)
                return
            for r in group[1:]:
                self.pending.remove(r)
            cap = max(r.nsteps for r in group)
            try:
                h = tb.tm_chain_begin_lanes(slot.handle, [r.iq for r in group], [r.direction for r in group],
                                            head.flavour, cap, stream=slot.stream.cuda_stream)
            except Exception:
                self.pool.release(nb)
                raise
            now = self.now()
            for r in group:
                r.t_admit = now
            slot.active.append(_Active(group, h, head.flavour, cap, 0, nb, [False] * len(group)))

    def _fail(self, req: Request, msg: str) -> None:
        req.error = msg
        req.chi = np.full((3, len(req.omega)), np.nan, dtype=np.complex128)
        req.t_admit = req.t_done = self.now()
        self.done.append(req)

    def _finish_lanes(self, a: _Active) -> None:
        """Finishes every request whose lane has run its steps."""
        lanes = None
        for i, r in enumerate(a.reqs):
            if a.done[i] or a.issued < r.nsteps:
                continue
            if lanes is None:
                lanes = tb.tm_chain_coeffs_lanes(a.chain, a.cap)
            _finish(r, lanes[i])
            r.t_done = self.now()
            a.done[i] = True
            self.done.append(r)

    def _end(self, slot: SystemSlot, a: _Active) -> None:
        tb.tm_chain_end(a.chain)
        self.pool.release(a.nbytes)

    def abort(self) -> None:
        """Ends every admitted chain and releases its memory (after an error)."""
        for slot in self.systems.values():
            for a in slot.active:
                try:
                    self._end(slot, a)
                except Exception:
                    pass
            slot.active = []

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
                    self._end(slot, a)
                else:
                    keep.append(a)
            slot.active = keep
            if slot.active:
                slot.last_used = time.perf_counter()

    def run(self, requests: List[Request]) -> List[Request]:
        """Replay requests at their arrival times (seconds from now); returns them completed."""
        todo = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        i = 0
        try:
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
        except BaseException:
            self.abort()
            raise
        return self.done

    def close(self) -> None:
        self.pool.close()


def _nelem_of_desc(d, iq: int) -> int:
    """Complex elements of a BR vector of q set iq, from a descriptor (tm_qset_info's nelem)."""
    roles = np.asarray(d.roles)
    nk = roles.shape[1]
    # every q set of a system pads its spheres to the longest of all of them
    npw = max(d.points[int(roles[jq, ik, 2])].mill.shape[0] for jq in range(roles.shape[0]) for ik in range(nk))
    return 2 * nk * d.nbnd * 2 * ((npw + 15) // 16 * 16)


def run_one_at_a_time(systems: Dict[str, SystemSlot], requests: List[Request], specs=None,
                      budget_bytes: int = 0) -> List[Request]:
    """Reference path: FIFO, one request at a time, every kernel issued directly
    (no graphs); spec systems are created and evicted under the same budget."""
    import torch
    pool = SystemPool(systems, budget_bytes or (1 << 62), specs)
    tb.tm_chains_use_graphs(False)
    try:
        t0 = time.perf_counter()
        for req in sorted(requests, key=lambda r: r.arrival):
            now = time.perf_counter() - t0
            if req.arrival > now:
                time.sleep(req.arrival - now)
            req.t_admit = time.perf_counter() - t0
            nb = chain_bytes(pool.systems[req.system].nelem[req.iq] if req.system in pool.systems
                             else _nelem_of_desc(pool.desc(req.system), req.iq), req.flavour, req.nsteps)
            try:
                slot = pool.acquire(req.system, nb)
                err = None if slot is not None else "does not fit the device-memory budget"
            except tb.TmError as e:
                slot, err = None, f"system cannot be created: {e}"
            if slot is None:
                req.error = err
                req.chi = np.full((3, len(req.omega)), np.nan, dtype=np.complex128)
            else:
                try:
                    co = tb.tm_lanczos_run(slot.handle, req.iq, req.direction, req.flavour, req.nsteps)
                    _finish(req, co)
                finally:
                    pool.release(nb)
            torch.cuda.synchronize()
            req.t_done = time.perf_counter() - t0
    finally:
        tb.tm_chains_use_graphs(True)
        pool.close()
    return requests


def summary(reqs: List[Request]) -> dict:
    lat = np.array([r.t_done - r.arrival for r in reqs])
    span = max(r.t_done for r in reqs) - min(r.arrival for r in reqs)
    ok = [r for r in reqs if r.coeffs is not None]
    return {"spectra_per_s": round(len(reqs) / span, 4), "p50_s": round(float(np.percentile(lat, 50)), 4),
            "p99_s": round(float(np.percentile(lat, 99)), 4), "requests": len(reqs),
            "steps": int(sum(r.coeffs["steps_done"] for r in ok)),
            "breakdowns": int(sum(bool(r.coeffs["breakdown"]) for r in ok)),
            "failed": int(sum(r.error is not None and r.coeffs is None for r in reqs))}
