"""Serving form: a continuous-batching request loop over aggregation rounds.

Each request is one Lancelot round (Algorithm 1, Server Executes): n clients'
packed, encrypted updates whose pairwise squared distances the KGC needs.
Rounds differ in client count, model size and ring degree.  The loop

  * admits arrived rounds in arrival order whenever a stream slot is free and
    the round's HBM footprint fits the budget (admission control);
  * runs every admitted round on a stream of its own: its packed
    ciphertexts are produced (device encryption of the clients' encoded
    chunks) and folded into the lazy triples k-chunk by k-chunk, so a round
    larger than the budget still runs (Methods, Lazy Relinearization: the
    triples of all k are summed before the one relinearization); then one
    relinearization per pair, rotate-and-sum, and the KGC's decryption;
  * polls completion events without blocking, frees slots and memory as
    rounds finish, and admits the next -- requests that arrive while others
    are on the GPU join as capacity frees up, and their kernels overlap on
    the device (one context per ring degree: resident keys and tables are
    shared, scratch memory is per stream).

The scheduling core (`Scheduler`) is plain Python with no GPU dependency so
that its admission logic is testable on the CPU; `GpuExecutor` drives the
C ABI.  All arithmetic happens in the HIP library.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Dict, List

import numpy as np


@dataclasses.dataclass
class RoundSpec:
    rid: int
    arrival: float        # seconds after the stream starts
    chain: str            # ring-degree parameter set name
    n: int                # clients
    dim: int              # model dimension
    n_byz: int
    attack: str           # "scale10" | "flip5" | "noise0.1"
    seed: int


@dataclasses.dataclass
class ChainInfo:
    name: str
    log_n: int
    nq: int
    np_: int
    scale_log2: int
    # context whose lc_footprint sizes the rounds (the server context, so
    # that its key-switch batch is the one counted); a host-only context of
    # the same shape is made on first use when none is given
    ctx: object = None

    def sizing_ctx(self):
        if self.ctx is None:
            from . import lancelot as L
            self.ctx = L.Context(self.log_n, (50,) * self.nq, (50,) * self.np_, device=-1)
        return self.ctx

    @property
    def N(self):
        return 1 << self.log_n

    @property
    def slots(self):
        return self.N // 2

    def n_ct(self, dim):
        return -(-dim // self.slots)

    def ct_bytes(self):
        return 2 * self.nq * self.N * 8


def round_footprint(ch: ChainInfo, n: int, dim: int, k_chunk: int) -> int:
    """Device bytes a round holds while admitted (lc_footprint): its client
    ciphertexts (all of them when they fit one k-chunk, else one chunk and
    the P lazy triples), their plaintexts, the P distance ciphertexts and
    their decryptions."""
    from . import lancelot as L
    rb, _ = ch.sizing_ctx().footprint(n, ch.n_ct(dim), k_chunk, L.FP_PLAINTEXTS | L.FP_DECRYPT)
    return rb


def stream_workspace(ch: ChainInfo, n_max: int, k_chunk: int) -> int:
    """Library workspace one stream can grow for rounds of up to n_max clients
    of a chain, resident (len <= k_chunk) or streamed (kept by the stream
    between rounds)."""
    from . import lancelot as L
    ctx = ch.sizing_ctx()
    return max(ctx.footprint(n_max, ln, k_chunk, L.FP_PLAINTEXTS | L.FP_DECRYPT)[1]
               for ln in (k_chunk, k_chunk + 1))


def make_stream(n_rounds: int, rate: float, chains: List[str], seed: int = 3000,
                clients=(5, 10, 20, 40), dims=(100_000, 1_000_000, 11_200_000)) -> List[RoundSpec]:
    """Poisson arrivals (rate per second) of rounds drawing client count,
    model size and ring degree uniformly; 10-20% Byzantine clients, at least
    one, with the attack cycling through the three workload attacks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    attacks = ("scale10", "flip5", "noise0.1")
    for r in range(n_rounds):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        n = int(rng.choice(clients))
        frac = rng.uniform(0.1, 0.2)
        out.append(RoundSpec(rid=r, arrival=t, chain=str(rng.choice(chains)), n=n, dim=int(rng.choice(dims)),
                             n_byz=max(1, int(round(frac * n))), attack=attacks[r % 3], seed=int(rng.integers(1 << 62))))
    return out


class Scheduler:
    """Admission and slot bookkeeping.  An executor provides
    start(spec) -> handle, poll(handle) -> bool (done), finish(handle)."""

    def __init__(self, chains: Dict[str, ChainInfo], budget_bytes: int, slots: int, k_chunk: int):
        self.chains = chains
        self.budget = budget_bytes
        self.slots = slots
        self.k_chunk = k_chunk
        self.used = 0
        self.deferred = 0  # admissions the executor put off for lack of device memory
        self.refused: List[int] = []  # rounds whose footprint alone exceeds the budget (not run)
        self.active: Dict[int, tuple] = {}

    def footprint(self, spec: RoundSpec) -> int:
        return round_footprint(self.chains[spec.chain], spec.n, spec.dim, self.k_chunk)

    def can_admit(self, spec: RoundSpec) -> bool:
        fp = self.footprint(spec)
        if fp > self.budget:
            raise ValueError("round %d needs %d bytes, more than the whole budget" % (spec.rid, fp))
        return len(self.active) < self.slots and self.used + fp <= self.budget

    def run(self, specs: List[RoundSpec], executor, clock: Callable[[], float] = time.perf_counter,
            sleep: Callable[[float], None] = time.sleep,
            on_done: Callable[[int, dict], None] = None) -> Dict[int, dict]:
        """Serve `specs` (sorted by arrival).  Returns per-round records with
        arrival, admit and completion times (seconds from the start);
        on_done(rounds_finished, record) is called as each round completes."""
        pending = sorted(specs, key=lambda s: s.arrival)
        waiting: List[RoundSpec] = []
        done: Dict[int, dict] = {}
        t0 = clock()
        i = 0
        while i < len(pending) or waiting or self.active:
            now = clock() - t0
            while i < len(pending) and pending[i].arrival <= now:
                waiting.append(pending[i])
                i += 1
            # admit in arrival order while capacity allows; an executor that
            # cannot place a round right now (start returns None) keeps it at
            # the head of the queue until a running round frees memory; a
            # round that could never fit the budget is refused, not run
            while waiting:
                if self.footprint(waiting[0]) > self.budget:
                    self.refused.append(waiting.pop(0).rid)
                    continue
                if not self.can_admit(waiting[0]):
                    break
                spec = waiting[0]
                handle = executor.start(spec)
                if handle is None:
                    if not self.active:
                        raise MemoryError("round %d (n=%d, dim=%d, %s; footprint %d bytes) cannot be placed even "
                                          "on an idle device: %s" % (spec.rid, spec.n, spec.dim, spec.chain,
                                                                     self.footprint(spec),
                                                                     getattr(executor, "last_refusal", None)))
                    self.deferred += 1
                    break
                waiting.pop(0)
                fp = self.footprint(spec)
                self.used += fp
                self.active[spec.rid] = (spec, handle, fp, clock() - t0)
            progressed = False
            for rid in list(self.active):
                spec, handle, fp, t_admit = self.active[rid]
                if executor.poll(handle):
                    result = executor.finish(handle)
                    t_done = clock() - t0
                    del self.active[rid]
                    self.used -= fp
                    done[rid] = {"rid": rid, "arrival": spec.arrival, "admit": t_admit, "done": t_done,
                                 "latency": t_done - spec.arrival, "chain": spec.chain, "n": spec.n, "dim": spec.dim,
                                 "result": result}
                    progressed = True
                    if on_done is not None:
                        on_done(len(done), done[rid])
            if not progressed:
                nxt = pending[i].arrival - (clock() - t0) if i < len(pending) else None
                if self.active or waiting:
                    sleep(0.0005)
                elif nxt is not None and nxt > 0:
                    sleep(min(nxt, 0.01))
        return done


def latency_stats(records: Dict[int, dict]) -> dict:
    """p50 / p99 / mean latency (arrival to completion), its split into
    queueing (arrival to admission) and service (admission to completion),
    rounds/s and client-pair distances/s over the span of the records."""
    recs = list(records.values())
    lat = np.array([r["latency"] for r in recs])
    queue = np.array([r["admit"] - r["arrival"] for r in recs])
    service = np.array([r["done"] - r["admit"] for r in recs])
    span = max(r["done"] for r in recs) - min(r["arrival"] for r in recs)
    pairs = sum(r["n"] * (r["n"] - 1) // 2 for r in recs)
    return {"rounds": len(lat), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "mean_queue_s": float(queue.mean()), "mean_service_s": float(service.mean()),
            "rounds_per_s": len(lat) / span if span > 0 else math.inf,
            "distances_per_s": pairs / span if span > 0 else math.inf}


def latency_by_class(records: Dict[int, dict]) -> dict:
    """latency_stats per (chain, clients, model dimension) class: the tail of
    a mixed stream is set by its largest rounds' service time."""
    classes: Dict[str, dict] = {}
    for rid, r in records.items():
        classes.setdefault("%s/n%d/dim%d" % (r["chain"], r["n"], r["dim"]), {})[rid] = r
    return {k: latency_stats(v) for k, v in sorted(classes.items())}


# --------------------------------------------------------------------------
# GPU executor
# --------------------------------------------------------------------------

class PlaintextPool:
    """Encoded chunks of seeded N(0, std^2) updates for one ring degree.  A
    round's client chunk k is pool entry index(round, client, k); the
    Byzantine attacks scale the integer plaintext (x10, x-5) or draw from a
    second pool of N(0, 0.1^2) chunks.  The last packed ciphertext of a model
    uses a copy of the entry with the slots past the model's end zeroed.
    Keeping a pool bounds host encoding work; every round still gets fresh
    encryption randomness."""

    def __init__(self, torch, ctx, size: int, std: float, seed: int, scale: float, tails=()):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.slots = ctx.N // 2
        self.values = rng.normal(0.0, std, size=(size, self.slots))
        self.noise = rng.normal(0.0, 0.1, size=(size, self.slots))
        self.size = size
        self._enc = lambda z: ctx.encode(z, scale)  # noqa: E731
        self._torch = torch
        self.m = self._upload(self.values)
        self.m_noise = self._upload(self.noise)
        self.tails = {}
        for t in tails:
            self.add_tail(t)

    def _upload(self, vals):
        return self._torch.from_numpy(np.stack([self._enc(z) for z in vals])).cuda()

    def add_tail(self, t: int):
        if t and t not in self.tails:
            self.tails[t] = (self._upload(self.values[:, :t]), self._upload(self.noise[:, :t]))

    def index(self, spec: RoundSpec, client: int, k0: int, k: int):
        base = (spec.seed * 2654435761 + client * 40503) % self.size
        return [(base + 97 * kk) % self.size for kk in range(k0, k0 + k)]

    def reference_update(self, spec: RoundSpec, client: int, n_ct: int) -> np.ndarray:
        """The FP64 update a client's ciphertexts encode (for checks)."""
        idx = self.index(spec, client, 0, n_ct)
        byz = client >= spec.n - spec.n_byz
        src = self.noise if (byz and spec.attack == "noise0.1") else self.values
        u = src[idx].reshape(-1)[: spec.dim]
        if byz and spec.attack == "scale10":
            u = 10 * u
        elif byz and spec.attack == "flip5":
            u = -5 * u
        return u


def reference_distances(spec: RoundSpec, pool: PlaintextPool, n_ct: int) -> np.ndarray:
    U = np.stack([pool.reference_update(spec, i, n_ct) for i in range(spec.n)])
    g = U @ U.T
    d = np.diag(g)
    return np.array([d[i] + d[j] - 2 * g[i, j] for i in range(spec.n) for j in range(i + 1, spec.n)])


class GpuExecutor:
    """Runs each admitted round on a stream of its own through the C ABI."""

    def __init__(self, torch, contexts: Dict[str, tuple], pools: Dict[str, PlaintextPool],
                 chains: Dict[str, ChainInfo], plans: Dict[str, list], k_chunk: int, streams: int,
                 keep_ciphertexts: bool = False):
        self.torch = torch
        self.contexts = contexts        # chain -> (kgc ctx, server ctx)
        self.pools = pools
        self.chains = chains
        self.plans = plans
        self.k_chunk = k_chunk
        self.free_streams = [torch.cuda.Stream() for _ in range(streams)]
        self.pending = {}
        self.last_refusal = None
        # a finished round's result holds its distance ciphertexts on the
        # device only when asked (tests compare them); otherwise its memory
        # goes back to the pool as soon as the KGC's read-out is done
        self.keep_ciphertexts = keep_ciphertexts

    def _plaintexts(self, spec, pool, ch, k0, k):
        """[n][k][N] encoded plaintexts of chunk k0..k0+k of every client."""
        torch = self.torch
        ln = ch.n_ct(spec.dim)
        tail = spec.dim - (ln - 1) * ch.slots
        rows = []
        for i in range(spec.n):
            byz = i >= spec.n - spec.n_byz
            noise = byz and spec.attack == "noise0.1"
            idx = pool.index(spec, i, k0, k)
            full = pool.m_noise if noise else pool.m
            if k0 + k == ln and tail < ch.slots:  # last chunk holds the model's end
                pool.add_tail(tail)
                last = pool.tails[tail][1 if noise else 0]
                parts = [full.index_select(0, torch.tensor(idx[:-1], device="cuda"))] if k > 1 else []
                parts.append(last.index_select(0, torch.tensor(idx[-1:], device="cuda")))
                r = torch.cat(parts)
            else:
                r = full.index_select(0, torch.tensor(idx, device="cuda"))
            if byz and spec.attack == "scale10":
                r = r * 10
            elif byz and spec.attack == "flip5":
                r = r * -5
            rows.append(r)
        return torch.stack(rows).contiguous()

    def start(self, spec: RoundSpec):
        """Enqueue a round; None if the device cannot hold it right now (the
        scheduler retries once a running round has finished)."""
        for attempt in range(2):
            try:
                return self._start(spec)
            except Exception as e:  # device memory pressure
                if "allocation" not in str(e) and "out of memory" not in str(e):
                    raise
                free, total = self.torch.cuda.mem_get_info()
                self.last_refusal = ("%s | device free %.1f of %.1f GiB, torch allocated %.1f GiB, reserved %.1f GiB"
                                     % (str(e).splitlines()[0][:200], free / 2 ** 30, total / 2 ** 30,
                                        self.torch.cuda.memory_allocated() / 2 ** 30,
                                        self.torch.cuda.memory_reserved() / 2 ** 30))
                if attempt == 0:  # release torch's cached blocks of finished rounds and retry once
                    self.torch.cuda.synchronize()
                    self.torch.cuda.empty_cache()
        return None

    def _start(self, spec: RoundSpec):
        stream = self.free_streams.pop()
        try:
            return self._enqueue(spec, stream)
        except Exception:
            self.free_streams.append(stream)
            raise

    def _enqueue(self, spec: RoundSpec, stream):
        torch = self.torch
        ch = self.chains[spec.chain]
        kgc, srv = self.contexts[spec.chain]
        pool = self.pools[spec.chain]
        n, P, ln = spec.n, spec.n * (spec.n - 1) // 2, ch.n_ct(spec.dim)
        with torch.cuda.stream(stream):
            if ln <= self.k_chunk:
                # resident: every packed ciphertext of the round on the device,
                # then the batched pipeline in one call
                m = self._plaintexts(spec, pool, ch, 0, ln)
                cts = srv.encrypt(m.view(n * ln, ch.N), seed=spec.seed, first_object=0, stream=stream)
                del m
                dist = srv.pairwise_sqdist(cts.view(n, ln, 2, ch.nq, ch.N), plan=self.plans[spec.chain],
                                           stream=stream)
                del cts
            else:
                # streamed in chunks of k_chunk packed ciphertexts folded into
                # the lazy triples (the same residues: modular sums are exact)
                trip = torch.zeros((P, 3, ch.nq, ch.N), dtype=torch.int64, device="cuda")
                for k0 in range(0, ln, self.k_chunk):
                    k = min(self.k_chunk, ln - k0)
                    m = self._plaintexts(spec, pool, ch, k0, k)
                    # PRNG objects n k0 .. n (k0 + k) - 1: distinct for every (chunk, client, k)
                    cts = srv.encrypt(m.view(n * k, ch.N), seed=spec.seed, first_object=n * k0, stream=stream)
                    srv.pair_triples_acc(cts.view(n, k, 2, ch.nq, ch.N), trip, stream=stream)
                    del m, cts
                dist = srv.pairwise_finish(trip, n, plan=self.plans[spec.chain], stream=stream)
                del trip
            dec = kgc.decrypt(dist, stream=stream)
            coeff0 = dec[:, :, 0].contiguous()
            ev = torch.cuda.Event()
            ev.record(stream)
        return {"spec": spec, "stream": stream, "event": ev, "dist": dist, "coeff0": coeff0}

    def poll(self, h) -> bool:
        return h["event"].query()

    def finish(self, h):
        spec = h["spec"]
        kgc, _ = self.contexts[spec.chain]
        ch = self.chains[spec.chain]
        c0 = h["coeff0"].cpu().numpy().view(np.uint64).T.copy()
        d = kgc.crt_to_double(c0) / 2.0 ** (2 * ch.scale_log2)
        self.free_streams.append(h["stream"])
        out = {"distances": d}
        if self.keep_ciphertexts:
            out["dist_ct"] = h["dist"]
        h.clear()
        return out
