"""Host logic of the continuous-batching server (paper_2203_01120_amd.serving)
without a GPU: the library binding and torch's stream/event calls are
replaced by a fake that keeps chains as plain counters and returns
coefficients that depend only on (system, q set, direction, flavour, step).

What this checks is the scheduler's bookkeeping, which the GPU tests cover
only on the few mixes they run:
* every request gets its own lane's coefficients, cut to its own step count,
  whichever chain and lane it shared (so chi equals the one-at-a-time path);
* the device-memory budget is never exceeded at any create or chain begin,
  spec systems are created on demand and evicted least recently used first,
  and the budget returns to the caller's systems' footprint at the end;
* lanes are formed only from one system and flavour, step counts within the
  slack, one q set unless the system is resident, at most `lanes` of them,
  and at most `max_chains` chains run per system;
* a chain that breaks down before its first step finishes with an error and
  chi = 0 without calling the chi solver, one that breaks down later gets
  chi from the steps it ran, and a request that can never fit fails without
  blocking the queue;
* an error inside a round ends every admitted chain before it propagates.
"""
import hashlib
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2203_01120_amd import serving as sv

GB = 1 << 30


class FakeLib:
    """Stands in for paper_2203_01120_amd.binding: systems and chains as host
    records, coefficients from a hash of the lane's identity."""

    class TmError(RuntimeError):
        def __init__(self, code, msg):
            super().__init__(f"libtm error {code}: {msg}")
            self.code = code

    def __init__(self):
        self.specs = {}            # system name -> parameters
        self.systems = {}          # handle -> dict(name, limit, stepped)
        self.chains = {}           # handle -> dict(sys, lanes, cap, steps)
        self.next = 1000
        self.pool = None           # the SystemPool under test, for the budget check
        self.max_used = 0
        self.begins = []           # (system name, lane count, q sets)
        self.max_active = {}
        self.graphs = []
        self.fail_step_after = None

    # ---- set-up of fake systems --------------------------------------------
    def add(self, name, nk, nbnd, npw, nq=1, tables=1 * GB, resident=4 * GB, columns=2 * GB, ws=1 * GB,
            breakdown=None, refused=False, create_fails=False):
        """breakdown: {(iq, direction, flavour): step at which that lane stops};
        refused: the library refuses the system (as for an unsupported grid);
        create_fails: its footprint is known but creation fails (out of memory)"""
        pts = [SimpleNamespace(mill=np.zeros((npw, 3), dtype=int)) for _ in range(nq + 1)]
        roles = np.zeros((nq, nk, 4), dtype=int)
        for jq in range(nq):
            roles[jq, :, 2] = jq + 1
        desc = SimpleNamespace(name=name, xq=np.zeros((nq, 3)), roles=roles, points=pts, nbnd=nbnd)
        self.specs[name] = dict(nelem=2 * nk * nbnd * 2 * ((npw + 15) // 16 * 16), nq=nq,
                                mem=dict(tables=tables, resident_full=resident, columns_full=columns,
                                         workspace_per_rhs=ws),
                                breakdown=dict(breakdown or {}), refused=refused, create_fails=create_fails)
        return desc

    def _check_budget(self):
        if self.pool is not None:
            assert self.pool.used <= self.pool.budget, (self.pool.used, self.pool.budget)
            self.max_used = max(self.max_used, self.pool.used)

    # ---- system calls ------------------------------------------------------------
    def tm_system_create(self, d):
        if self.specs[d.name]["refused"]:
            raise self.TmError(-5, "FFT length must factor into 2, 3, 5")
        if self.specs[d.name]["create_fails"]:
            raise self.TmError(-2, "device allocation failed")
        self._check_budget()
        self.next += 1
        self.systems[self.next] = dict(name=d.name, limit=-1, stepped=False)
        return self.next

    def tm_system_destroy(self, h):
        assert not any(c["sys"] == h for c in self.chains.values()), "system destroyed under a live chain"
        del self.systems[h]

    def tm_system_footprint(self, d):
        if self.specs[d.name]["refused"]:
            raise self.TmError(-5, "FFT length must factor into 2, 3, 5")
        return dict(self.specs[d.name]["mem"])

    def tm_system_memory(self, h):
        return dict(self.specs[self.systems[h]["name"]]["mem"])

    def tm_system_set_resident_limit(self, h, n):
        self.systems[h]["limit"] = n

    def tm_system_set_chain_slots(self, h, n):
        assert n >= 1

    def tm_system_resident_bytes(self, h):
        s = self.systems[h]
        return self.specs[s["name"]]["mem"]["resident_full"] if s["stepped"] and s["limit"] != 0 else 0

    def tm_qset_info_get(self, h, iq):
        sp = self.specs[self.systems[h]["name"]]
        assert 0 <= iq < sp["nq"]
        return dict(nelem=sp["nelem"])

    def tm_chains_use_graphs(self, on):
        self.graphs.append(bool(on))

    # ---- coefficients ------------------------------------------------------------
    def _lane_limit(self, name, iq, d, flav):
        return self.specs[name]["breakdown"].get((iq, d, flav), 1 << 30)

    @staticmethod
    def _series(name, iq, d, flav, n):
        seed = int(hashlib.sha256(f"{name}/{iq}/{d}/{flav}".encode()).hexdigest()[:8], 16)
        rng = np.random.default_rng(seed)
        m = 4096                              # a lane's step j has one value, whatever the capacity
        a = rng.standard_normal(m) + 1j * rng.standard_normal(m)
        b = rng.uniform(0.5, 1.5, m)
        z = rng.standard_normal((3, m)) + 1j * rng.standard_normal((3, m))
        return a[:n], b[:n], z[:, :n]

    def _coeffs(self, name, iq, d, flav, cap, done, broke):
        a, b, z = self._series(name, iq, d, flav, cap)
        mask = np.arange(cap) < done
        return dict(alpha=np.where(mask, a, 0), beta=np.where(mask, b, 0), gamma=np.where(mask, b, 0).astype(complex),
                    z=np.where(mask, z, 0), zn=np.zeros(cap, complex), n1=float(len(name)), steps_done=done,
                    breakdown=broke)

    def tm_lanczos_run(self, h, iq, d, flav, nsteps):
        name = self.systems[h]["name"]
        self.systems[h]["stepped"] = True
        lim = self._lane_limit(name, iq, d, flav)
        done = min(nsteps, lim)
        return self._coeffs(name, iq, d, flav, nsteps, done, done < nsteps)

    def tm_chi(self, co, m_use, omega, eta):
        if not 1 <= m_use <= co["steps_done"]:
            raise RuntimeError(f"TM_EINVAL: m_use {m_use} with {co['steps_done']} steps done")
        w = np.arange(1, m_use + 1)
        base = np.sum(co["alpha"][:m_use] * w) + np.sum(co["beta"][:m_use]) * 1j + co["n1"]
        zs = np.sum(co["z"][:, :m_use], axis=1)
        return (base + zs)[:, None] * (1.0 + 0.0j) + 1j * eta * np.asarray(omega)[None, :]

    # ---- chains ------------------------------------------------------------------
    def tm_chain_begin_lanes(self, h, iqs, dirs, flav, cap, stream=None):
        self._check_budget()
        s = self.systems[h]
        assert len(iqs) == len(dirs) >= 1
        if len(set(iqs)) > 1:
            assert self.tm_system_resident_bytes(h) > 0, "lanes of different q sets on a non-resident system"
        self.next += 1
        self.chains[self.next] = dict(sys=h, lanes=[(iq, d, flav) for iq, d in zip(iqs, dirs)], cap=cap,
                                      steps=[0] * len(iqs), broke=[False] * len(iqs))
        self.begins.append((s["name"], len(iqs), tuple(iqs), flav))
        n = sum(c["sys"] == h for c in self.chains.values())
        self.max_active[s["name"]] = max(self.max_active.get(s["name"], 0), n)
        return self.next

    def tm_chains_step(self, chains, k, stream=None):
        if self.fail_step_after is not None:
            self.fail_step_after -= 1
            if self.fail_step_after < 0:
                raise RuntimeError("planted step failure")
        for ch in chains:
            c = self.chains[ch]
            name = self.systems[c["sys"]]["name"]
            self.systems[c["sys"]]["stepped"] = True
            for i, (iq, d, flav) in enumerate(c["lanes"]):
                lim = self._lane_limit(name, iq, d, flav)
                c["steps"][i] = min(c["cap"], c["steps"][i] + k, lim)
                c["broke"][i] = c["steps"][i] == lim and lim < c["cap"]

    def tm_chain_coeffs_lanes(self, ch, cap):
        c = self.chains[ch]
        assert cap == c["cap"]
        name = self.systems[c["sys"]]["name"]
        return [self._coeffs(name, iq, d, flav, cap, c["steps"][i], c["broke"][i])
                for i, (iq, d, flav) in enumerate(c["lanes"])]

    def tm_chain_end(self, ch):
        del self.chains[ch]


class _Stream:
    n = 0

    def __init__(self, *a, **k):
        _Stream.n += 1
        self.cuda_stream = _Stream.n


class _Event:
    def __init__(self, *a, **k):
        pass

    def record(self, stream=None):
        pass

    def synchronize(self):
        pass

    def elapsed_time(self, other):
        return 1.0


@pytest.fixture
def fake(monkeypatch):
    import torch
    lib = FakeLib()
    monkeypatch.setattr(sv, "tb", lib)
    monkeypatch.setattr(torch.cuda, "Stream", _Stream)
    monkeypatch.setattr(torch.cuda, "Event", _Event)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    return lib


OMEGA = np.linspace(0.0, 1.0, 7)


def _req(rid, system, iq, d, flav, n):
    return sv.Request(rid=rid, system=system, iq=iq, direction=d, flavour=flav, nsteps=n, omega=OMEGA,
                      eta=0.01, arrival=0.0)


def _copy(reqs):
    return [_req(r.rid, r.system, r.iq, r.direction, r.flavour, r.nsteps) for r in reqs]


def _server(fake, slots, budget, specs=None, **kw):
    srv = sv.Server(slots, budget, specs=specs, **kw)
    fake.pool = srv.pool
    return srv


def test_each_request_gets_its_own_lane(fake):
    """A mix that forms multi-lane chains (same system and flavour, step
    counts within the slack) and single chains: each request's coefficients
    and chi equal the one-at-a-time path's exactly."""
    d_a = fake.add("A", nk=2, nbnd=4, npw=100, nq=2)
    d_b = fake.add("B", nk=1, nbnd=8, npw=300)
    slots = {"A": sv.SystemSlot(handle=fake.tm_system_create(d_a), nelem={0: fake.specs["A"]["nelem"],
                                                                         1: fake.specs["A"]["nelem"]}),
             "B": sv.SystemSlot(handle=fake.tm_system_create(d_b), nelem={0: fake.specs["B"]["nelem"]})}
    reqs = [_req(0, "A", 0, "+", "pH", 40), _req(1, "A", 0, "-", "pH", 36), _req(2, "B", 0, "z", "nH", 20),
            _req(3, "A", 0, "z", "pH", 44), _req(4, "A", 0, "x", "pH", 12), _req(5, "B", 0, "+", "nH", 18),
            _req(6, "A", 1, "+", "pH", 40), _req(7, "A", 0, "y", "nH", 30)]
    srv = _server(fake, slots, 64 * GB, lanes=4)
    base = srv.used
    out = {r.rid: r for r in srv.run(_copy(reqs))}
    assert sorted(out) == list(range(len(reqs)))
    assert srv.used == base
    ref = {r.rid: r for r in sv.run_one_at_a_time(slots, _copy(reqs))}
    for rid, r in out.items():
        assert r.error is None
        assert r.coeffs["steps_done"] == r.nsteps and not r.coeffs["breakdown"]
        for k in ("alpha", "beta", "gamma", "z"):
            assert r.coeffs[k].shape[-1] == r.nsteps
            np.testing.assert_array_equal(r.coeffs[k], ref[rid].coeffs[k])
        np.testing.assert_array_equal(r.chi, ref[rid].chi)
        assert r.t_admit <= r.t_done
    # requests 0, 1, 3 share a chain (40, 36, 44 steps within 25 %); 4 (12 steps) does not
    lanes = sorted(b[1] for b in fake.begins if b[0] == "A" and b[3] == "pH")
    assert max(lanes) == 3 and 1 in lanes
    for name, n, iqs, flav in fake.begins:
        assert n <= 4
    assert not fake.chains


def test_lanes_respect_slack_flavour_and_q_sets(fake):
    """Lanes of different q sets only once the system is resident; other
    flavours and step counts beyond the slack never share a chain."""
    d = fake.add("A", nk=1, nbnd=4, npw=64, nq=3)
    slot = sv.SystemSlot(handle=fake.tm_system_create(d), nelem={i: fake.specs["A"]["nelem"] for i in range(3)})
    reqs = [_req(0, "A", 0, "+", "pH", 30), _req(1, "A", 1, "+", "pH", 30), _req(2, "A", 2, "-", "pH", 30),
            _req(3, "A", 0, "z", "nH", 30), _req(4, "A", 0, "x", "pH", 60)]
    srv = _server(fake, {"A": slot}, 64 * GB, lanes=4)
    srv.run(_copy(reqs))
    # nothing was resident at the first admission: one chain per q set
    first = [b for b in fake.begins if b[3] == "pH"]
    assert all(len(set(b[2])) == 1 for b in first)
    assert all(b[1] == 1 for b in fake.begins if b[3] == "nH")
    # the 60-step request never shares with a 30-step one (slack 1.25)
    # resident now: the next mix of q sets forms one chain
    fake.begins.clear()
    srv.run(_copy(reqs[:3]))
    assert fake.begins == [("A", 3, (0, 1, 2), "pH")]
    assert not fake.chains


def test_budget_creates_and_evicts_spec_systems(fake):
    """A budget that holds one spec system at a time: requests that alternate
    between two spec systems create and evict them; the budget is never
    exceeded and returns to zero after close."""
    da = fake.add("S1", nk=2, nbnd=4, npw=100, tables=1 * GB, resident=20 * GB, columns=2 * GB, ws=1 * GB)
    db = fake.add("S2", nk=2, nbnd=4, npw=100, tables=1 * GB, resident=20 * GB, columns=2 * GB, ws=1 * GB)
    specs = {"S1": sv.SystemSpec(make_desc=lambda: da, resident_cap=8 * GB),
             "S2": sv.SystemSpec(make_desc=lambda: db, resident_cap=-1)}
    budget = 26 * GB
    srv = _server(fake, {}, budget, specs=specs, lanes=1)
    # S1: resident copy (20 GB) above its 8 GB cap -> columns only: 1 + 2 + 1 GB
    assert srv.pool.footprint("S1") == 4 * GB
    # S2: resident within the budget: 1 + 20 + 2 + 1 GB
    assert srv.pool.footprint("S2") == 24 * GB
    reqs = [_req(i, "S1" if i % 2 == 0 else "S2", 0, "+-zxy"[i % 5], "pH", 18) for i in range(6)]
    ref = {r.rid: r for r in sv.run_one_at_a_time({}, _copy(reqs), specs=specs, budget_bytes=budget)}
    fake.max_used = 0
    fake.pool = srv.pool
    out = srv.run(_copy(reqs))
    assert len(out) == 6 and all(r.error is None for r in out)
    for r in out:
        np.testing.assert_array_equal(r.chi, ref[r.rid].chi)
    assert fake.max_used <= budget
    assert srv.pool.created >= 2 and srv.pool.evicted >= 1
    srv.close()
    assert srv.used == 0 and not fake.systems and not fake.chains


def test_breakdowns_and_requests_that_never_fit(fake):
    """Breakdown before the first step: error, chi = 0, no chi solve (the fake
    solver raises for m_use = 0). Breakdown at step 5 of 24: chi from 5
    steps. A request larger than the budget fails at once and the others run."""
    d = fake.add("T", nk=1, nbnd=3, npw=64, tables=1 * GB, resident=1 * GB, columns=1 * GB, ws=1 * GB,
                 breakdown={(0, "x", "pH"): 0, (0, "-", "nH"): 5})
    dbig = fake.add("BIG", nk=1, nbnd=3, npw=64, tables=100 * GB)
    specs = {"BIG": sv.SystemSpec(make_desc=lambda: dbig)}
    slot = sv.SystemSlot(handle=fake.tm_system_create(d), nelem={0: fake.specs["T"]["nelem"]})
    reqs = [_req(0, "T", 0, "x", "pH", 30), _req(1, "BIG", 0, "+", "pH", 10), _req(2, "T", 0, "-", "nH", 24),
            _req(3, "T", 0, "+", "pH", 30)]
    srv = _server(fake, {"T": slot}, 16 * GB, specs=specs, lanes=4)
    base = srv.used
    out = {r.rid: r for r in srv.run(_copy(reqs))}
    g = out[0]
    assert g.coeffs["steps_done"] == 0 and g.coeffs["breakdown"] and g.error
    assert np.all(g.chi == 0)
    big = out[1]
    assert big.error and big.coeffs is None and np.all(np.isnan(big.chi))
    b5 = out[2]
    assert b5.coeffs["steps_done"] == 5 and b5.coeffs["breakdown"] and b5.error is None
    np.testing.assert_array_equal(b5.chi, fake.tm_chi(b5.coeffs, 5, OMEGA, 0.01))
    assert out[3].error is None and out[3].coeffs["steps_done"] == 30
    assert srv.used == base and not fake.chains
    st = sv.summary(list(out.values()))
    assert st["requests"] == 4 and st["failed"] == 1 and st["breakdowns"] == 2
    assert st["p50_s"] <= st["p99_s"]


def test_chain_limit_per_system(fake):
    """max_chains = 2: never more than two chains of one system at a time;
    the waiting requests run later (as lanes once they pile up)."""
    d = fake.add("A", nk=1, nbnd=4, npw=64)
    slot = sv.SystemSlot(handle=fake.tm_system_create(d), nelem={0: fake.specs["A"]["nelem"]})
    reqs = [_req(i, "A", 0, "+-zxy"[i % 5], "pH" if i < 5 else "nH", 12 + 6 * (i % 4)) for i in range(10)]
    srv = _server(fake, {"A": slot}, 64 * GB, lanes=2, max_chains=2)
    base = srv.used
    out = srv.run(_copy(reqs))
    assert len(out) == 10 and all(r.error is None for r in out)
    assert fake.max_active["A"] <= 2
    assert all(b[1] <= 2 for b in fake.begins)
    assert not fake.chains and srv.used == base


def test_error_in_a_round_ends_every_chain(fake):
    """A failure inside tm_chains_step propagates out of Server.run after
    every admitted chain is ended and its memory released."""
    d = fake.add("A", nk=1, nbnd=4, npw=64)
    slot = sv.SystemSlot(handle=fake.tm_system_create(d), nelem={0: fake.specs["A"]["nelem"]})
    reqs = [_req(i, "A", 0, "+-z"[i % 3], "pH", 60 + 20 * i) for i in range(3)]
    srv = _server(fake, {"A": slot}, 64 * GB, lanes=1)
    base = srv.used
    fake.fail_step_after = 2
    with pytest.raises(RuntimeError, match="planted"):
        srv.run(_copy(reqs))
    assert not fake.chains and srv.used == base


def test_a_system_the_library_refuses_fails_only_its_requests(fake):
    """A spec system whose footprint query (and creation) the library refuses,
    as for a grid length with a prime factor other than 2, 3, 5, and one whose
    creation fails (out of device memory) after its footprint was admitted:
    their requests finish with an error and chi = NaN, nothing stays charged,
    and the other requests run, in the server and one at a time alike."""
    d = fake.add("A", nk=1, nbnd=4, npw=64)
    dbad = fake.add("BAD", nk=1, nbnd=4, npw=64, refused=True)
    doom = fake.add("OOM", nk=1, nbnd=4, npw=64, create_fails=True)
    specs = {"BAD": sv.SystemSpec(make_desc=lambda: dbad), "OOM": sv.SystemSpec(make_desc=lambda: doom)}
    slot = sv.SystemSlot(handle=fake.tm_system_create(d), nelem={0: fake.specs["A"]["nelem"]})
    reqs = [_req(0, "BAD", 0, "+", "pH", 12), _req(1, "A", 0, "+", "pH", 12), _req(2, "OOM", 0, "z", "nH", 6),
            _req(3, "A", 0, "z", "nH", 9), _req(4, "OOM", 0, "+", "nH", 6)]
    srv = _server(fake, {"A": slot}, 64 * GB, specs=specs, lanes=2)
    base = srv.used
    out = {r.rid: r for r in srv.run(_copy(reqs))}
    ref = {r.rid: r for r in sv.run_one_at_a_time({"A": slot}, _copy(reqs), specs=specs, budget_bytes=64 * GB)}
    for res in (out, ref):
        for rid in (0, 2, 4):
            assert "cannot be created" in res[rid].error and np.all(np.isnan(res[rid].chi))
        for rid in (1, 3):
            assert res[rid].error is None and res[rid].coeffs["steps_done"] == reqs[rid].nsteps
    np.testing.assert_array_equal(out[1].chi, ref[1].chi)
    assert srv.used == base and not fake.chains
