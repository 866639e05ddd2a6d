"""Benchmark: encrypted client-pair squared distances per second on one MI355X.

One step = one pass of the server's hot path over one round of resident
client ciphertexts: fused subtract/square/lazy-accumulate over all pairs and
packed ciphertexts, one relinearization per pair, rotate-and-sum (block plan
of hoisted rotations), SumDis, the plaintext-mask aggregation of every
client ciphertext, and the KGC's decryption of the distance ciphertexts.
Ingest (device FP64 encode + device encryption) happens before the timed
region and is reported separately.

Prints one JSON line (see --help for options).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# rounds of very different sizes share the device in the serving form:
# growable segments keep torch's cache from fragmenting (set before torch loads)
os.environ.setdefault("PYTORCH_ALLOC_CONF", "expandable_segments:True")

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, vendor figure
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # FP64 lane-instructions/s: 256 CUs x 4 SIMD16 x 2.4 GHz (78.6 TFLOP/s)
A2_OPS_PER_UPDATE = 23

# HBM traffic of the pair-triple kernel from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE) of `python -m paper_2408_06197_amd.profile_cases
# pair`, each scaled by what the counter reads for a 4 GiB device copy
# (FETCH_SIZE 2.0x low, WRITE_SIZE exact); see
# profiles/pair_triples_n65536_l24_20clients_pmc.txt.  Valid only for the
# kernel source it was taken on: the section of ops.hip is hashed at run time.
A2_PMC = {"fetch_bytes": 2.0 * 84056392 * 1024, "write_bytes": 7004160 * 1024,
          "source_sha256": "3844a40c5187beb1493f22bd107fa53f981d017b1b830998616b543e8387f78d"}
A2_SECTION = ("ops.hip", "// ---- fused subtract / square / lazy accumulate over all pairs", "// ---- SumDis[i]")
# The same for the forward NTT's two launches on 64 ciphertexts' limbs
# (1536 limb-polynomials at N = 2^16): `python -m
# paper_2408_06197_amd.profile_cases ntt`, per-launch averages of the forward
# passes; see profiles/ntt_fwd_n65536_l24_64cts_pmc.txt.  Empty until taken.
NTT_SECTION = ("ntt.hip", "// ---- register-radix pass kernel", "struct FastPass {")
NTT_PMC = {"fetch_bytes_per_launch": 2.0 * (393379 + 399428) / 2 * 1024, "write_bytes_per_launch": 786432 * 1024,
           "limb_polys": 1536,
           "source_sha256": "94e0ef1e433c0177aac1b0d213d016d4572cdb4b1810e0552cc6d4398501ffbf"}


def _source_sha256(fname, start, stop):
    import hashlib
    src = open(os.path.join(ROOT, "paper_2408_06197_amd", "csrc", fname)).read()
    a = src.index(start)
    b = src.index(stop)
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser(description=__doc__)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="cfg3", choices=["cfg1", "cfg2", "cfg3"])
    p.add_argument("--plan", default=None, help="rotate-sum block plan, e.g. 2,2,2,2,2,2,2,1 (default: autotuned)")
    p.add_argument("--no-tune", dest="tune", action="store_false", default=True,
                   help="skip the launch-shape / plan autotuner")
    p.add_argument("--cpu-baseline", dest="cpu_baseline", action="store_true", default=True)
    p.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    p.add_argument("--per-op-pairs", type=int, default=2, help="pairs timed in the plain per-op form (0: skip)")
    p.add_argument("--no-graph", dest="graph", action="store_false", default=True,
                   help="time eager launches instead of a captured HIP graph")
    p.add_argument("--no-round", dest="round", action="store_false", default=True,
                   help="skip the selection / encrypted-mask aggregation / model decryption of the round")
    p.add_argument("--no-ablation", dest="ablation", action="store_false", default=True,
                   help="skip the lazy/eager relinearization and per-client SumDis ablations")
    p.add_argument("--no-ntt-micro", dest="ntt_micro", action="store_false", default=True,
                   help="skip the mixed-degree NTT / hoisted key-switch micro-workload")
    p.add_argument("--serve", type=int, default=100, metavar="ROUNDS",
                   help="serving form: ROUNDS Poisson-arriving aggregation rounds (0: skip)")
    p.add_argument("--no-small-configs", dest="small_configs", action="store_false", default=True,
                   help="skip the N=2^12 and N=2^14 workloads (batched, per-op and eager forms)")
    p.add_argument("--serve-slots", type=int, default=4)
    p.add_argument("--sweep-n", dest="sweep_n", action="store_true", default=False,
                   help="also run the packing-size sweep N = 2^13..2^17 on the depth-3 parameters")
    p.add_argument("--stages", action="store_true", default=True, help="time each stage with events")
    p.add_argument("--no-stages", dest="stages", action="store_false")
    return p.parse_args()


def fp64_pair_distances(upd):
    g = upd @ upd.T
    n = upd.shape[0]
    d = np.diag(g)
    return np.array([d[i] + d[j] - 2 * g[i, j] for i in range(n) for j in range(i + 1, n)])


def event_time(torch, fn, reps=1):
    """Average milliseconds of fn() on torch's current stream."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def ntt_roofline(torch, srv, batch):
    """Forward NTT of `batch` ciphertext-sized blocks (batch x n_q limb-polys),
    the shape the key-switch stages transform.  Returns per-launch figures:
    two launches (passes) per transform, each with 8 N bytes of algorithmic
    traffic per limb-polynomial (the transform's one read plus one write,
    16 N bytes, split over its two launches)."""
    import synth
    x = synth.device_residues_mod(torch, 1717, srv.q, (batch, srv.nq, srv.N))
    s = torch.cuda.current_stream()
    ms = event_time(torch, lambda: srv.ntt_fwd(x, nlimb=srv.nq, stream=s), reps=5)
    npoly = batch * srv.nq
    launches = 2
    per_launch_ms = ms / launches
    bytes_per_launch = 8 * srv.N * npoly
    del x
    return {"launch_ms": per_launch_ms, "bytes_per_launch": bytes_per_launch, "limb_polys": npoly,
            "transform_ms_per_limb_poly": ms / npoly}


# ---- mixed-degree NTT and hoisted key-switch micro-workload --------------------
# 4096 single-limb polynomials of mixed ring degree in ratio 4:2:1, on one
# chain of 50-bit primes = 1 mod 2^17 (NTT-friendly for every degree): poly i
# of a degree uses limb prime i mod (L+1) of that degree's chain.  The key
# switch groups consecutive polynomials of a degree into RNS c1's with
# (L+1, K = alpha) = (3,1) / (6,2) / (24,8), so dnum = 3 for all three.
D4 = ((12, 2341, 3, 1), (14, 1170, 6, 2), (16, 585, 24, 8))  # (log N, polys, L+1, K)


def d4_contexts(L):
    return [L.Context(ln, (50,) * nq, (50,) * k, log_m=17, device=0, role=L.ROLE_KGC) for ln, _, nq, k in D4]


def d4_polys(torch, ctxs, seed):
    """Per degree: (full groups [g][L+1][N], ragged tail [1][r][N] or None),
    coefficients uniform in [0, q) of each poly's prime."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    out = []
    for ctx, (_, cnt, nq, _) in zip(ctxs, D4):
        full, rem = divmod(cnt, nq)
        x = torch.empty((full, nq, ctx.N), dtype=torch.int64, device="cuda")
        for l in range(nq):
            x[:, l].random_(0, int(ctx.moduli[l]), generator=gen)
        y = None
        if rem:
            y = torch.empty((1, rem, ctx.N), dtype=torch.int64, device="cuda")
            for l in range(rem):
                y[:, l].random_(0, int(ctx.moduli[l]), generator=gen)
        out.append((x, y))
    return out


def d4_ntt(ctxs, polys, inverse=False):
    """One context per degree, two launches per degree and tail."""
    for ctx, (x, y) in zip(ctxs, polys):
        f = ctx.ntt_inv if inverse else ctx.ntt_fwd
        f(x, nlimb=x.shape[1])
        if y is not None:
            f(y, nlimb=y.shape[1])


def d4_groups(polys):
    """The micro-workload as polynomial groups of one mixed-degree call."""
    g = []
    for (x, y), (ln, _, nq, _) in zip(polys, D4):
        g.append((x, ln, nq, 0))
        if y is not None:
            g.append((y, ln, y.shape[1], 0))
    return g


def d4_ntt_mixed(big, polys, inverse=False):
    """All 4096 polynomials in one launch per pass on the degree-2^16 context
    (whose chain starts with the smaller degrees' primes)."""
    (big.ntt_inv_groups if inverse else big.ntt_fwd_groups)(d4_groups(polys))


def d4_rotation_steps(log_n):
    return [1 << j for j in range(log_n - 1)]


def ntt_micro(torch, L):
    """Forward + inverse NTT of the 4096 mixed-degree polys (checked to round
    trip), then one hoisted key switch per c1 over log2(N/2) power-of-two
    rotations.  Algorithmic NTT traffic: one read + one write of every poly
    per direction (16 N bytes per poly)."""
    ctxs = d4_contexts(L)
    polys = d4_polys(torch, ctxs, 4004)
    keep = [(x.clone(), None if y is None else y.clone()) for x, y in polys]
    alg_bytes = sum(cnt * (1 << ln) * 16 for ln, cnt, _, _ in D4)
    res = {"polys": {str(1 << ln): cnt for ln, cnt, _, _ in D4}, "algorithmic_bytes_per_direction": alg_bytes}
    # one launch per pass over every polynomial of every degree (the
    # degree-2^16 context's chain starts with the smaller contexts' primes)
    big = ctxs[-1]
    assert big.moduli[:3] == ctxs[0].moduli[:3] and big.moduli[:6] == ctxs[1].moduli[:6]
    fwd = event_time(torch, lambda: d4_ntt_mixed(big, polys), reps=3)
    inv = event_time(torch, lambda: d4_ntt_mixed(big, polys, inverse=True), reps=3)
    # the same transforms as per-degree launches (six calls of two passes)
    res["per_degree_fwd_ms"] = event_time(torch, lambda: d4_ntt(ctxs, polys), reps=3)
    res["per_degree_inv_ms"] = event_time(torch, lambda: d4_ntt(ctxs, polys, inverse=True), reps=3)
    torch.cuda.synchronize()
    # the timed transforms ran in forward/inverse pairs: the data is back
    res["round_trip_exact"] = all(bool(torch.equal(x, a)) and (y is None or bool(torch.equal(y, b)))
                                  for (x, y), (a, b) in zip(polys, keep))
    # and the mixed call gives the per-degree contexts' bits
    d4_ntt_mixed(big, polys)
    ref = [(x.clone(), None if y is None else y.clone()) for x, y in keep]
    d4_ntt(ctxs, ref)
    res["mixed_equals_per_degree"] = all(bool(torch.equal(x, a)) and (y is None or bool(torch.equal(y, b)))
                                         for (x, y), (a, b) in zip(polys, ref))
    d4_ntt_mixed(big, polys, inverse=True)
    del ref
    res.update({"launches_per_direction": 2, "fwd_ms": fwd, "inv_ms": inv,
                "fwd_GBps": alg_bytes / (fwd / 1e3) / 1e9, "inv_GBps": alg_bytes / (inv / 1e3) / 1e9})
    log(f"[bench] NTT micro (2341x2^12 + 1170x2^14 + 585x2^16, one launch per pass): fwd {fwd:.2f} ms "
        f"({res['fwd_GBps']:.0f} GB/s), inv {inv:.2f} ms ({res['inv_GBps']:.0f} GB/s); per-degree launches "
        f"{res['per_degree_fwd_ms']:.2f} / {res['per_degree_inv_ms']:.2f} ms; round trip "
        f"{'exact' if res['round_trip_exact'] else 'MISMATCH'}, mixed == per-degree: {res['mixed_equals_per_degree']}")
    del keep
    ks = {}
    for ctx, (x, _), (ln, cnt, nq, k) in zip(ctxs, polys, D4):
        steps = d4_rotation_steps(ln)
        ctx.keygen(4104)
        ctx.keygen_rotation(4104, steps)
        g = x.shape[0]
        ct = torch.empty((g, 2, nq, ctx.N), dtype=torch.int64, device="cuda")
        ct[:, 1].copy_(x)
        ct[:, 0].copy_(x.flip(0))
        out = torch.empty((g, len(steps), 2, nq, ctx.N), dtype=torch.int64, device="cuda")
        ms = event_time(torch, lambda: ctx.rotate_hoisted(ct, steps, out=out), reps=2)
        key_bytes = ctx.dnum * 2 * (nq + k) * ctx.N * 8
        # algorithmic: read c1 once and c0 per step, keys once per call, write every output
        alg = g * (nq * ctx.N * 8 * (1 + len(steps)) + len(steps) * 2 * nq * ctx.N * 8) + len(steps) * key_bytes
        ks[str(1 << ln)] = {"c1": g, "limbs": nq, "special": k, "dnum": ctx.dnum, "rotations": len(steps),
                            "ms": ms, "rotations_per_s": g * len(steps) / (ms / 1e3),
                            "algorithmic_GBps": alg / (ms / 1e3) / 1e9}
        log(f"[bench] hoisted KS 2^{ln}: {g} c1 x {len(steps)} rotations in {ms:.1f} ms "
            f"({ks[str(1 << ln)]['algorithmic_GBps']:.0f} GB/s algorithmic)")
        del ct, out
    res["hoisted_keyswitch"] = ks
    del polys
    return res


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def _omp_threads(k):
    """Thread count of the oracle's OpenMP regions (libgomp, as the oracle is
    built with gcc -fopenmp); None if it cannot be set."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))
        return int(k)
    except OSError:
        return None


def _oracle_keys(O, w, plan):
    ora = O.Oracle(w.log_n, w.q_bits, w.p_bits)
    s = ora.secret(w.crypto_seed)
    rlk = ora.relin_key(w.crypto_seed, s)
    rks = [ora.rot_key(w.crypto_seed, s, k) for k in ora.rotsum_steps(plan)]
    return ora, s, rlk, rks


def _oracle_pair(ora, cts, rlk, plan, rks):
    """Times (tensor phase, relinearization, rotate-and-sum) of one pair."""
    t0 = time.perf_counter()
    tri = ora.pair_triple(cts, 0, 1)
    t1 = time.perf_counter()
    d = ora.relin(tri, rlk)
    t2 = time.perf_counter()
    ora.rotate_sum(d, plan, rks)
    t3 = time.perf_counter()
    return t1 - t0, t2 - t1, t3 - t2


def cpu_baseline(w, plan, small_plans):
    """The oracle on the host cores (all of them, then one thread on a
    sample), reported as client-pair distances/s:
      * the N = 2^16 workload: one whole client pair -- the tensor phase over
        all LEN packed ciphertexts, one relinearization and the rotate-and-sum
        with the bench's plan -- with no scaling; the inputs are synthetic
        residues (16 random packed ciphertexts per client repeated to LEN:
        the oracle's work does not depend on the values);
      * one thread: the same pair's relinearization and the tensor phase over
        16 packed ciphertexts, against the same sample on all threads;
      * the N = 2^12 and N = 2^14 workloads in full (every pair, real
        encryptions), distances checked against FP64.
    Key generation is set-up and is not timed."""
    from oracle import oracle as O
    import synth

    cpu = host_cpu()
    threads = _omp_threads(cpu["nproc"])
    ora, s, rlk, rks = _oracle_keys(O, w, plan)
    block = synth.uniform_residues(77, ora.q, (2, 16, 2, w.N))
    cts = np.empty((2, w.n_ct) + block.shape[2:], dtype=np.uint64)
    for k0 in range(0, w.n_ct, 16):
        k = min(16, w.n_ct - k0)
        cts[:, k0:k0 + k] = block[:, :k]
    del block
    t_tensor, t_relin, t_rot = _oracle_pair(ora, cts, rlk, plan, rks)
    sec = t_tensor + t_relin + t_rot
    # one thread against all threads on a sample of the same pair
    sample = np.ascontiguousarray(cts[:, :16])
    del cts
    t_all = sum(_oracle_pair(ora, sample, rlk, plan, rks)[:2])
    one = _omp_threads(1)
    t_one = sum(_oracle_pair(ora, sample, rlk, plan, rks)[:2]) if one else None
    _omp_threads(cpu["nproc"])
    del sample
    full = {}
    for sw, pl in small_plans:
        t0 = time.perf_counter()
        o2, s2, rlk2, rks2 = _oracle_keys(O, sw, pl)
        pk2 = o2.pk(sw.crypto_seed, s2)
        upd = synth.client_updates(sw)
        scale = 2.0 ** sw.scale_log2
        m = np.stack([np.stack([O.encode(c, sw.log_n, scale) for c in synth.pack(u, sw.slots)]) for u in upd])
        n, ln = m.shape[:2]
        c2 = o2.encrypt(sw.crypto_seed + 1, 0, m.reshape(n * ln, sw.N), pk2).reshape(n, ln, 2, o2.nq, sw.N)
        t_setup = time.perf_counter() - t0
        t1 = time.perf_counter()
        res = o2.pairwise(c2, rlk2, pl, rks2, want_sumdis=False)
        t_run = time.perf_counter() - t1
        got = np.array([o2.read_distance(o2.decrypt(d, s2), scale * scale) for d in res["dist"]])
        ref = fp64_pair_distances(upd)
        full[sw.name] = {"pairs": sw.n_pairs, "plan": pl, "seconds": t_run, "distances_per_s": sw.n_pairs / t_run,
                         "setup_s_untimed": t_setup,
                         "max_rel_err_vs_fp64": float(np.max(np.abs(got - ref) / np.abs(ref)))}
        log(f"[bench] oracle {sw.name}: {sw.n_pairs} pairs in {t_run:.1f}s ({sw.n_pairs / t_run:.2f} distances/s)")
    return {"value": 1.0 / sec, "unit": "client-pair distances/s", "cores": threads or cpu["nproc"],
            "kind": "oracle",
            "sample": "one whole client pair of the %s workload, not scaled: tensor phase over all %d packed "
                      "ciphertexts (%.1f s), one relinearization (%.1f s), rotate-and-sum with plan %s (%.1f s); "
                      "synthetic residues (16 random packed ciphertexts per client repeated to %d)"
                      % (w.name, w.n_ct, t_tensor, t_relin, ",".join(map(str, plan)), t_rot, w.n_ct),
            "seconds_per_pair": sec, "cpu": cpu,
            "one_thread": {"sample": "tensor phase over 16 packed ciphertexts + one relinearization",
                           "seconds": t_one, "seconds_all_threads": t_all,
                           "speedup_all_threads": (t_one / t_all) if t_one else None},
            "full_configs": full}


def plans_for(log_n):
    levels = log_n - 1
    return [[1] * levels, [2] * (levels // 2) + [1] * (levels % 2), [3] * (levels // 3) + ([levels % 3] if levels % 3 else [])]


def graph_form(torch, fn, outs, pairs):
    """fn (library calls on torch's current stream) captured into a HIP graph
    on a stream of its own after a warm-up call there has grown that stream's
    workspaces; three replays, with eager work between them, must equal the
    eager result before the replays are timed."""
    sg = torch.cuda.Stream()
    res = {"ms": None, "replays_equal_eager": False}
    with torch.cuda.stream(sg):
        fn()
        sg.synchronize()
        want = [t.clone() for t in outs]
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=sg):
                fn()
            ok = True
            for rep in range(3):
                if rep == 1:
                    fn()
                for t in outs:
                    t.fill_(-1)
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                ok &= all(bool(torch.equal(a, b)) for a, b in zip(outs, want))
            res["replays_equal_eager"] = ok
            if ok:
                ms = event_time(torch, g.replay, reps=10)
                res.update({"ms": ms, "distances_per_s": pairs / (ms / 1e3)})
            del g
        except Exception as e:  # capture is optional; the eager figure stands
            res["error"] = str(e)
    torch.cuda.synchronize()
    return res


def small_config(torch, L, synth, w):
    """A smaller workload at full size on the GPU, in every form: device
    ingest; the batched pipeline (lc_pairwise_sqdist) under each hoisting
    plan; the plain per-op launch form over every pair (lc_ct_sub,
    lc_ct_square and lc_ct_add per packed ciphertext, then lc_relin and
    lc_rotate_sum per pair); the eager-relinearization form (a
    relinearization per packed ciphertext, Table 2's "without lazy
    relinearization"); per-client SumDis (lc_sumdis_lazy).  Every form's
    decrypted distances are checked against FP64."""
    n, ln, N, P = w.n_clients, w.n_ct, w.N, w.n_pairs
    scale = 2.0 ** w.scale_log2
    plans = plans_for(w.log_n)
    kgc = L.Context(w.log_n, w.q_bits, w.p_bits, device=0, role=L.ROLE_KGC)
    srv = L.Context(w.log_n, w.q_bits, w.p_bits, device=0, role=L.ROLE_SERVER)
    kgc.keygen(w.crypto_seed)
    kgc.keygen_rotation(w.crypto_seed, sorted({s_ for pl in plans for s_ in kgc.rotsum_steps(pl)}))
    kgc.keys_share(srv)
    upd = synth.client_updates(w)
    ref = fp64_pair_distances(upd)
    nq = srv.nq
    cts = torch.empty((n, ln, 2, nq, N), dtype=torch.int64, device="cuda")
    for i in range(n):
        z = torch.from_numpy(synth.pack(upd[i], w.slots)).cuda()
        srv.encrypt(srv.encode_device(z, scale), seed=w.crypto_seed + 1, first_object=i * ln, out=cts[i])
    dist = torch.empty((P, 2, nq, N), dtype=torch.int64, device="cuda")

    def rel_err(d):
        dec = kgc.decrypt(d)[:, :, 0].cpu().numpy().view(np.uint64).T.copy()
        got = kgc.crt_to_double(dec) / scale ** 2
        return float(np.max(np.abs(got - ref) / np.abs(ref)))

    res = {"N": N, "limbs": nq, "clients": n, "ciphertexts_per_client": ln, "pairs": P}
    best = None
    for pl in plans:
        ms = event_time(torch, lambda: srv.pairwise_sqdist(cts, plan=pl, out=dist), reps=3)
        res.setdefault("batched_ms_by_plan", {})[",".join(map(str, pl))] = ms
        if best is None or ms < best[0]:
            best = (ms, pl)
    ms, plan = best
    srv.pairwise_sqdist(cts, plan=plan, out=dist)
    res["batched"] = {"plan": plan, "ms": ms, "distances_per_s": P / (ms / 1e3), "max_rel_err_vs_fp64": rel_err(dist)}
    res["batched_graph"] = graph_form(torch, lambda: srv.pairwise_sqdist(cts, plan=plan, out=dist), [dist], P)
    pidx = [(a, b) for a in range(n) for b in range(a + 1, n)]
    tmp = torch.empty((1, 2, nq, N), dtype=torch.int64, device="cuda")
    sq = torch.empty((1, 3, nq, N), dtype=torch.int64, device="cuda")
    acc3 = torch.empty((1, 3, nq, N), dtype=torch.int64, device="cuda")
    acc2 = torch.empty((1, 2, nq, N), dtype=torch.int64, device="cuda")
    r2 = torch.empty((1, 2, nq, N), dtype=torch.int64, device="cuda")
    out = torch.empty((P, 2, nq, N), dtype=torch.int64, device="cuda")

    def per_op(eager):
        for p_, (a, b) in enumerate(pidx):
            (acc2 if eager else acc3).zero_()
            for k in range(ln):
                srv.ct_sub(cts[a, k], cts[b, k], out=tmp)
                srv.ct_square(tmp, out=sq)
                if eager:
                    srv.relin(sq, out=r2)
                    srv.ct_add(acc2, r2, out=acc2)
                else:
                    srv.ct_add(acc3, sq, out=acc3, ncomp=3)
            if eager:
                out[p_].copy_(acc2[0])
            else:
                srv.relin(acc3, out=out[p_:p_ + 1])
            srv.rotate_sum(out[p_:p_ + 1], plan)

    for name, eager in (("per_op_lazy", False), ("per_op_eager", True)):
        t = event_time(torch, lambda: per_op(eager))
        res[name] = {"ms": t, "distances_per_s": P / (t / 1e3), "max_rel_err_vs_fp64": rel_err(out),
                     "key_switches_per_pair": (ln if eager else 1) + len(plan)}
    res["lazy_vs_eager_speedup"] = res["per_op_eager"]["ms"] / res["per_op_lazy"]["ms"]
    res["batched_vs_per_op_speedup"] = res["per_op_lazy"]["ms"] / res["batched"]["ms"]
    sd = torch.empty((n, 2, nq, N), dtype=torch.int64, device="cuda")
    t_sd = event_time(torch, lambda: srv.sumdis_lazy(cts, plan=plan, out=sd), reps=3)
    dec = kgc.decrypt(sd)[:, :, 0].cpu().numpy().view(np.uint64).T.copy()
    D = np.zeros((n, n))
    for p_, (a, b) in enumerate(pidx):
        D[a, b] = D[b, a] = ref[p_]
    got = kgc.crt_to_double(dec) / scale ** 2
    res["sumdis_per_client"] = {"ms": t_sd, "key_switch_chains": n,
                                "max_rel_err_vs_fp64": float(np.max(np.abs(got - D.sum(1)) / D.sum(1)))}
    gf = res["batched_graph"]
    if gf.get("ms"):
        log(f"[bench] {w.name}: batched as a HIP graph {gf['ms']:.3f} ms ({gf['distances_per_s']:.0f} distances/s, "
            f"replays equal the eager result: {gf['replays_equal_eager']})")
    log(f"[bench] {w.name}: batched {ms:.2f} ms ({P / (ms / 1e3):.0f} distances/s, plan {plan}); per-op "
        f"{res['per_op_lazy']['ms']:.1f} ms, eager relin {res['per_op_eager']['ms']:.1f} ms "
        f"({res['lazy_vs_eager_speedup']:.1f}x); max rel err {res['batched']['max_rel_err_vs_fp64']:.1e}")
    del cts, dist, out, sd
    for c in (srv, kgc):
        c.release_workspace()
    return res


def sweep_n(torch, L, synth, log_ns=(13, 14, 15, 16, 17), dim=11_200_000, n=20, steps=2):
    """Packing-size sweep (a Fig. 3 analog): the paper's default depth-3
    parameters (Delta = 2^40; Q = 50 + 3 x 40 bits, one 48-bit special prime:
    218 bits, inside the 128-bit bound at N = 2^13) at N = 2^13 .. 2^17, the
    same model (n clients x `dim` parameters) packed into N/2 slots per
    ciphertext.  Per N: device ingest, then the timed round (all pairs'
    distances with SumDis, the masked sum, decryption), checked against FP64."""
    res = []
    for log_n in log_ns:
        w = synth.Workload(f"depth3_n{1 << log_n}", log_n, (50, 40, 40, 40), (48,), 40, n, dim, 0.005, 4, "scale10",
                           data_seed=101, crypto_seed=202)
        N, ln, P = w.N, w.n_ct, w.n_pairs
        levels = log_n - 1
        plan = [3] * (levels // 3) + ([levels % 3] if levels % 3 else [])
        scale = 2.0 ** w.scale_log2
        t0 = time.perf_counter()
        kgc = L.Context(log_n, w.q_bits, w.p_bits, device=0, role=L.ROLE_KGC)
        srv = L.Context(log_n, w.q_bits, w.p_bits, device=0, role=L.ROLE_SERVER)
        kgc.keygen(w.crypto_seed)
        kgc.keygen_rotation(w.crypto_seed, kgc.rotsum_steps(plan))
        kgc.keys_share(srv)
        nq = srv.nq
        cts = torch.empty((n, ln, 2, nq, N), dtype=torch.int64, device="cuda")
        upd_all = np.empty((n, dim), dtype=np.float64)
        for i in range(n):
            upd_all[i] = synth.client_updates(w, clients=[i])[0]
            z = torch.from_numpy(synth.pack(upd_all[i], w.slots)).cuda()
            srv.encrypt(srv.encode_device(z, scale), seed=w.crypto_seed + 1, first_object=i * ln, out=cts[i])
            del z
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        ref = fp64_pair_distances(upd_all)
        del upd_all
        dist = torch.empty((P, 2, nq, N), dtype=torch.int64, device="cuda")
        sumdis = torch.empty((n, 2, nq, N), dtype=torch.int64, device="cuda")
        agg = torch.empty((ln, 2, nq, N), dtype=torch.int64, device="cuda")
        dec = torch.empty((P, nq, N), dtype=torch.int64, device="cuda")
        masks = torch.zeros((n, nq, N), dtype=torch.int64, device="cuda")
        masks[0].fill_(1)

        def step():
            srv.pairwise_sqdist(cts, plan=plan, sumdis=True, out=dist, sumdis_out=sumdis)
            srv.masked_sum(cts, masks, out=agg)
            kgc.decrypt(dist, out=dec)

        step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / steps
        got = kgc.crt_to_double(dec[:, :, 0].cpu().numpy().view(np.uint64).T.copy()) / scale ** 2
        rel = float(np.max(np.abs(got - ref) / np.abs(ref)))
        rec = {"N": N, "ciphertexts_per_client": ln, "plan": plan, "ms_per_round": ms,
               "distances_per_s": P / (ms / 1e3), "setup_s": t_setup, "max_rel_err_vs_fp64": rel}
        res.append(rec)
        log(f"[bench] sweep N=2^{log_n}: {ln} cts/client, plan {','.join(map(str, plan))}: {ms:.1f} ms/round, "
            f"{P / (ms / 1e3):.1f} distances/s, max rel err {rel:.1e} (setup {t_setup:.1f}s)")
        del cts, dist, sumdis, agg, dec, masks
        srv.release_workspace()
        kgc.release_workspace()
        del srv, kgc
        torch.cuda.empty_cache()
    return res


def serve_bench(args, torch, L, srv16, kgc16, plan16):
    """Serving form: Poisson stream of aggregation rounds over the N=2^14
    (8 limbs) and N=2^16 (24 limbs) parameter sets, 5..40 clients, 1e5..1.12e7
    dims, continuous admission by HBM footprint; returns rounds/s, p50, p99."""
    from paper_2408_06197_amd import serve
    import synth

    w14, w16 = synth.CFG2, synth.CFG3
    kgc14 = L.Context(w14.log_n, w14.q_bits, w14.p_bits, device=0, role=L.ROLE_KGC)
    srv14 = L.Context(w14.log_n, w14.q_bits, w14.p_bits, device=0, role=L.ROLE_SERVER)
    # rounds are sized by lc_footprint of the server contexts
    chains = {"n16384_l8": serve.ChainInfo("n16384_l8", 14, 8, 2, 40, ctx=srv14),
              "n65536_l24": serve.ChainInfo("n65536_l24", 16, 24, 4, 40, ctx=srv16)}
    plan14 = [3] * 4 + [1]
    kgc14.keygen(w14.crypto_seed)
    kgc14.keygen_rotation(w14.crypto_seed, kgc14.rotsum_steps(plan14))
    kgc14.keys_share(srv14)
    contexts = {"n16384_l8": (kgc14, srv14), "n65536_l24": (kgc16, srv16)}
    plans = {"n16384_l8": plan14, "n65536_l24": plan16}
    k_chunk = 32
    for c in (srv14, srv16):
        c.set_tuning("ks_chunk", 32)
    t0 = time.perf_counter()
    pools = {}
    for name, ch in chains.items():
        ctx = contexts[name][1]
        tails = sorted({d - (ch.n_ct(d) - 1) * ch.slots for d in (100_000, 1_000_000, 11_200_000)})
        pools[name] = serve.PlaintextPool(torch, ctx, size=64, std=0.01, seed=3001, scale=2.0 ** ch.scale_log2,
                                          tails=[t for t in tails if t < ch.slots])
    log(f"[bench] serving: pools encoded in {time.perf_counter() - t0:.1f}s")
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    # large frees can reach the free-memory count a little later: take the
    # largest of a few readings
    free = 0
    for _ in range(5):
        free = max(free, torch.cuda.mem_get_info()[0])
        time.sleep(0.1)
    # leave room for the library's per-stream workspace (the largest a stream
    # can grow for 40-client rounds, lc_footprint) and for torch's cache
    ws = max(serve.stream_workspace(ch, 40, k_chunk) for ch in chains.values())
    budget = int(0.5 * (free - args.serve_slots * ws))
    log(f"[bench] serving: {free / 1e9:.1f} GB free, {args.serve_slots} slots x {ws / 1e9:.1f} GB stream "
        f"workspace, admission budget {budget / 1e9:.1f} GB")
    names = list(chains)

    def progress(k, rec):
        if k % 25 == 0:
            log(f"[bench] serving: {k} rounds done (last: n={rec['n']} dim={rec['dim']} {rec['chain']}, "
                f"latency {rec['latency']:.3f}s)")

    refused = []

    def run(specs):
        ex = serve.GpuExecutor(torch, contexts, pools, chains, plans, k_chunk=k_chunk, streams=args.serve_slots)
        sch = serve.Scheduler(chains, budget, slots=args.serve_slots, k_chunk=k_chunk)
        rec = sch.run(specs, ex, on_done=progress)
        refused.extend(sch.refused)
        return rec

    # closed-loop calibration: a burst of 24 rounds arriving together (the
    # class mix of a shorter burst, and with it the capacity, varied from run
    # to run)
    calib = serve.make_stream(24, rate=0.0, chains=names, seed=2999)
    t0 = time.perf_counter()
    rec = run(calib)
    torch.cuda.synchronize()
    capacity = len(calib) / (time.perf_counter() - t0)
    rate = 0.7 * capacity
    del rec
    torch.cuda.empty_cache()
    log(f"[bench] serving: closed-loop capacity {capacity:.2f} rounds/s; Poisson rate {rate:.2f}/s")
    specs = serve.make_stream(args.serve, rate=rate, chains=names, seed=3000)
    t0 = time.perf_counter()
    refused.clear()
    rec = run(specs)
    wall = time.perf_counter() - t0
    st = serve.latency_stats(rec)
    st["refused_rounds"] = list(refused)  # footprint above the whole admission budget: not run
    if refused:
        log(f"[bench] serving: {len(refused)} rounds refused (footprint above the budget): {refused}")
    # every tenth round's decrypted distances against FP64
    errs = []
    for rid in sorted(r for r in rec if r % 10 == 0):
        sp = specs[rid]
        ref = serve.reference_distances(sp, pools[sp.chain], chains[sp.chain].n_ct(sp.dim))
        got = rec[rid]["result"]["distances"]
        errs.append(float(np.max(np.abs(got - ref) / np.abs(ref))))
    by_class = serve.latency_by_class(rec)
    # the rounds behind the tail: the slowest 2% and their classes
    slow = sorted(rec.values(), key=lambda r: -r["latency"])[: max(1, len(rec) // 50)]
    st.update({"wall_s": wall, "slots": args.serve_slots, "k_chunk": k_chunk, "budget_bytes": budget,
               "stream_workspace_bytes": ws, "rate_per_s": rate, "calibrated_capacity_per_s": capacity,
               "checked_rounds": len(errs), "max_rel_err_vs_fp64": max(errs) if errs else None,
               "resident_rounds": sum(1 for r in rec.values() if chains[r["chain"]].n_ct(r["dim"]) <= k_chunk),
               "by_chain": {c: serve.latency_stats({k: v for k, v in rec.items() if v["chain"] == c})
                            for c in names if any(v["chain"] == c for v in rec.values())},
               "by_class": by_class,
               "slowest": [{"rid": r["rid"], "chain": r["chain"], "n": r["n"], "dim": r["dim"],
                            "latency_s": r["latency"], "queue_s": r["admit"] - r["arrival"],
                            "service_s": r["done"] - r["admit"]} for r in slow]})
    log(f"[bench] serving: {st['rounds']} rounds in {wall:.1f}s, {st['rounds_per_s']:.2f} rounds/s, "
        f"{st['distances_per_s']:.1f} distances/s, p50 {st['p50_s']:.3f}s p99 {st['p99_s']:.3f}s (mean queue "
        f"{st['mean_queue_s']:.3f}s, service {st['mean_service_s']:.3f}s), max rel err {st['max_rel_err_vs_fp64']}")
    for r in st["slowest"]:
        log(f"[bench] serving tail: round {r['rid']} {r['chain']} n={r['n']} dim={r['dim']}: "
            f"{r['latency_s']:.2f}s = queue {r['queue_s']:.2f}s + service {r['service_s']:.2f}s")
    return st


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: multi-GPU runs are not supported (the packed-ciphertext axis would "
              "shard across GPUs with one reduce-scatter of the triple accumulators).", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2408_06197_amd import lancelot as L

    w = synth.WORKLOADS[args.workload]
    levels = w.log_n - 1
    if args.plan:
        plans = [[int(x) for x in args.plan.split(",")]]
    else:  # dynamic hoisting: blocks of 1, 2 or 3 levels, chosen by measurement
        plans = [[1] * levels, [2] * (levels // 2) + [1] * (levels % 2), [3] * (levels // 3) + [1] * (levels % 3)]
    plan = plans[0]
    torch.cuda.set_device(0)
    # All library work of the bench runs on one non-default stream (HIP graph
    # capture needs one; the library keeps its workspaces per stream).
    s_main = torch.cuda.Stream()
    torch.cuda.set_stream(s_main)
    n, ln, N = w.n_clients, w.n_ct, w.N
    P = w.n_pairs
    scale = 2.0 ** w.scale_log2

    t_setup = time.perf_counter()
    kgc = L.Context(w.log_n, w.q_bits, w.p_bits, device=0, role=L.ROLE_KGC)
    srv = L.Context(w.log_n, w.q_bits, w.p_bits, device=0, role=L.ROLE_SERVER)
    kgc.keygen(w.crypto_seed)
    kgc.keygen_rotation(w.crypto_seed, sorted({s for pl in plans for s in kgc.rotsum_steps(pl)}))
    kgc.keys_share(srv)
    t_keys = time.perf_counter() - t_setup
    log(f"[bench] {w.name}: keys ready in {t_keys:.1f}s; ingesting {n} clients x {ln} ciphertexts")

    # ---- ingest: device encode and encryption (the host encoder is timed on
    # one client for comparison) ----------------------------------------------
    nq = srv.nq
    cts = torch.empty((n, ln, 2, nq, N), dtype=torch.int64, device="cuda")
    upd_all = np.empty((n, w.dim), dtype=np.float64)
    t_h2d = t_enc_dev = t_encrypt = 0.0
    host_cmp = {}
    for i in range(n):
        upd = synth.client_updates(w, clients=[i])[0]
        upd_all[i] = upd
        chunks = synth.pack(upd, w.slots)
        t0 = time.perf_counter()
        z_dev = torch.from_numpy(chunks).cuda()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m_dev = srv.encode_device(z_dev, scale)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        srv.encrypt(m_dev, seed=w.crypto_seed + 1, first_object=i * ln, out=cts[i])
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        t_h2d += t1 - t0
        t_enc_dev += t2 - t1
        t_encrypt += t3 - t2
        if i == 0:
            with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as pool:
                th = time.perf_counter()
                m_host = np.stack(list(pool.map(lambda c: srv.encode(c, scale), chunks)))
                host_cmp["encode_host_s_per_client"] = time.perf_counter() - th
            d = np.abs(m_dev.cpu().numpy() - m_host)
            host_cmp["max_coeff_diff"] = int(d.max())
            host_cmp["coeffs_differing"] = int(np.count_nonzero(d))
            del m_host, d
        del z_dev, m_dev
        if (i + 1) % 5 == 0 or i + 1 == n:
            log(f"[bench] ingested {i + 1}/{n} clients")
    ref = fp64_pair_distances(upd_all)
    del upd_all
    log(f"[bench] ingest: H2D {t_h2d:.2f}s, device encode {t_enc_dev:.2f}s, encrypt {t_encrypt:.2f}s; "
        f"host encode of one client {host_cmp['encode_host_s_per_client']:.2f}s (16 threads), device vs host "
        f"encode: max diff {host_cmp['max_coeff_diff']}, {host_cmp['coeffs_differing']} coefficients differ")

    # ---- buffers -----------------------------------------------------------------
    dist = torch.empty((P, 2, nq, N), dtype=torch.int64, device="cuda")
    sumdis = torch.empty((n, 2, nq, N), dtype=torch.int64, device="cuda")
    agg = torch.empty((ln, 2, nq, N), dtype=torch.int64, device="cuda")
    dec = torch.empty((P, nq, N), dtype=torch.int64, device="cuda")
    masks = torch.zeros((n, nq, N), dtype=torch.int64, device="cuda")
    masks[0].fill_(1)  # one-hot plaintext mask on client 0 (constant 1 in the NTT domain)

    # ---- autotuner: pair-kernel launch shape, then the hoisting plan -------------
    tuned = {}
    if args.tune:
        trip = torch.empty((P, 3, nq, N), dtype=torch.int64, device="cuda")
        best = None
        for lanes in (16, 32, 64):
            for ppt in (3, 4, 6):
                srv.set_tuning("pair_lanes", lanes)
                srv.set_tuning("pair_ppt", ppt)
                ms = event_time(torch, lambda: srv.pair_triples(cts, out=trip))
                tuned.setdefault("pair_kernel_ms", {})["%dx%d" % (lanes, ppt)] = ms
                if best is None or ms < best[0]:
                    best = (ms, lanes, ppt)
        srv.set_tuning("pair_lanes", best[1])
        srv.set_tuning("pair_ppt", best[2])
        tuned["pair_lanes"], tuned["pair_ppt"] = best[1], best[2]
        # the Gram form on the int8 matrix cores (4 coefficients per workgroup)
        srv.set_tuning("pair_mfma", 4)
        ms = event_time(torch, lambda: srv.pair_triples(cts, out=trip))
        tuned["pair_kernel_ms"]["gram_mfma_4"] = ms
        tuned["pair_mfma"] = 4 if ms < best[0] else 0
        srv.set_tuning("pair_mfma", tuned["pair_mfma"])
        del trip
        # hoisting plan jointly with the shortest tile cycle that the
        # cycle-walking inner product takes (2^30: never)
        bestp = None
        for pl in plans:
            for cmin in (1 << 30, 128, 16, 2):
                srv.set_tuning("mac_cycle_min", cmin)
                ms = event_time(torch, lambda: srv.pairwise_sqdist(cts, plan=pl, out=dist))
                tuned.setdefault("plan_ms", {})["%s/%d" % (",".join(map(str, pl)), cmin)] = ms
                if bestp is None or ms < bestp[0]:
                    bestp = (ms, pl, cmin)
        plan = bestp[1]
        srv.set_tuning("mac_cycle_min", bestp[2])
        tuned["plan"], tuned["mac_cycle_min"] = plan, bestp[2]
        # key-switch inner-product width and batch, on the chosen plan (the NTT
        # sub-batch knob measured no gain at this size and stays off)
        bestm = None
        for shp in (0, 1, 2):  # masked-sum lane shape
            srv.set_tuning("ms_shape", shp)
            ms = event_time(torch, lambda: srv.masked_sum(cts, masks, out=agg))
            tuned.setdefault("ms_shape_ms", {})[str(shp)] = ms
            if bestm is None or ms < bestm[0]:
                bestm = (ms, shp)
        srv.set_tuning("ms_shape", bestm[1])
        tuned["ms_shape"] = bestm[1]
        # (ks_chunk 192: every distance ciphertext in one key-switch batch, one
        # launch per stage; each trial starts from released workspaces, so
        # outgrown batches do not stay resident)
        for name, values in (("mac_cycle_short", (1, 0)), ("mac_cycle_cts", (8, 16)), ("mac_short_cts", (16, 8)),
                             ("mac_cycle_c0", (1, 0)),
                             ("mac_cts", (8, 16)),
                             ("ks_chunk", (32, 64, 128, 192)),
                             ("ks_streams", (2, 1))):
            bestv = None
            for v in values:
                if name in ("ks_chunk", "ks_streams"):
                    srv.release_workspace()
                srv.set_tuning(name, v)
                ms = event_time(torch, lambda: srv.pairwise_sqdist(cts, plan=plan, out=dist))
                tuned.setdefault(name + "_ms", {})[str(v)] = ms
                if bestv is None or ms < bestv[0]:
                    bestv = (ms, v)
            srv.set_tuning(name, bestv[1])
            tuned[name] = bestv[1]
        srv.release_workspace()
        log(f"[bench] autotuned: {tuned}")

    def step():
        srv.pairwise_sqdist(cts, plan=plan, sumdis=True, out=dist, sumdis_out=sumdis)
        srv.masked_sum(cts, masks, out=agg)
        kgc.decrypt(dist, out=dec)

    # With --graph (default) the step is captured once into a HIP graph and
    # replayed: after the warmup has grown the stream's workspaces the library
    # allocates, copies and synchronizes nothing inside it, and issues no memset.
    graph = None
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (dist, sumdis, agg, dec)]
    if args.graph:
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s_main):
                step()
            torch.cuda.synchronize()
            graph_ok = True
            for rep in range(3):
                # eager work and a synchronization between replays, then every
                # replay is compared with the eager result
                if rep == 1:
                    step()
                for t in (dist, sumdis, agg, dec):
                    t.fill_(-1)
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                graph_ok &= all(bool(torch.equal(a, b)) for a, b in zip((dist, sumdis, agg, dec), eager))
            if graph_ok:
                graph = g
            log(f"[bench] HIP graph capture {'verified on 3 replays' if graph_ok else 'MISMATCH: timing eager'}")
        except Exception as e:  # capture is optional; the eager path is the same work
            log(f"[bench] HIP graph capture unavailable ({e}); timing eager launches")
    del eager
    log(f"[bench] warmup done ({args.warmup} steps); timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / max(1, args.steps)
    value = P / (ms_per_step / 1e3)
    log(f"[bench] {ms_per_step:.1f} ms/step -> {value:.1f} distances/s")

    # ---- correctness of what was timed ------------------------------------------
    d0 = dec[:, :, 0].cpu().numpy().view(np.uint64).T.copy()
    got = kgc.crt_to_double(d0) / scale ** 2
    rel = np.abs(got - ref) / np.abs(ref)
    log(f"[bench] decrypted distances vs FP64: max rel err {rel.max():.2e} over {P} pairs")
    check = {"max_rel_err_vs_fp64": float(rel.max()), "pairs": P, "ok": bool(rel.max() < 1e-4)}

    # ---- the rest of the round (Algorithm 1: KGC selection and encrypted mask,
    # ServerUpdate): Multi-Krum on the decrypted distances, Enc_pk of each
    # client's weight 1/l (or 0) at scale Delta, the masked aggregation of all
    # packed ciphertexts with one relinearization each, and the KGC's
    # decryption of the aggregated model (first and last ciphertext checked
    # against the FP64 mean of the chosen updates)
    extra = {}
    if args.round:
        from paper_2408_06197_amd import robust
        t_sel0 = time.perf_counter()
        c_byz = w.n_byz
        chosen = robust.select("multikrum", robust.distance_matrix(got, n), c_byz, l=n - c_byz)
        t_sel = time.perf_counter() - t_sel0
        chosen_fp64 = robust.select("multikrum", robust.distance_matrix(ref, n), c_byz, l=n - c_byz)
        wts = robust.weights("multikrum", chosen, n)
        m_mask = torch.from_numpy(robust.mask_plaintexts(wts, N, scale)).cuda()
        mask_ct = torch.empty((n, 2, nq, N), dtype=torch.int64, device="cuda")
        t_mask = event_time(torch, lambda: kgc.encrypt(m_mask, seed=w.crypto_seed + 7, first_object=1 << 40,
                                                        out=mask_ct))
        agg2 = torch.empty((ln, 2, nq, N), dtype=torch.int64, device="cuda")
        t_agg = event_time(torch, lambda: srv.mask_aggregate(cts, mask_ct, out=agg2))
        dec_agg = torch.empty((ln, nq, N), dtype=torch.int64, device="cuda")
        t_dec_agg = event_time(torch, lambda: kgc.decrypt(agg2, out=dec_agg))
        errs = []
        for k in (0, ln - 1):
            z = kgc.decode(dec_agg[k].cpu().numpy().view(np.uint64), scale * scale).real
            lo, hi = k * w.slots, min((k + 1) * w.slots, w.dim)
            want = np.zeros(w.slots)
            for i in chosen:
                want[: hi - lo] += synth.client_updates(w, clients=[i])[0][lo:hi] / len(chosen)
            errs.append(float(np.max(np.abs(z - want))))
        del agg2, dec_agg, mask_ct, m_mask
        extra["round"] = {"rule": "multikrum", "c": c_byz, "l": n - c_byz, "chosen": chosen,
                          "same_as_fp64_selection": chosen == chosen_fp64,
                          "byzantine_chosen": int(sum(i >= n - c_byz for i in chosen)),
                          "kgc_select_ms": t_sel * 1e3, "mask_encrypt_ms": t_mask, "mask_aggregate_ms": t_agg,
                          "decrypt_model_ms": t_dec_agg, "max_abs_err_vs_fp64_mean": max(errs),
                          "update_std": w.std}
        log(f"[bench] round: Multi-Krum chose {len(chosen)} clients ({extra['round']['byzantine_chosen']} "
            f"Byzantine; same as FP64: {chosen == chosen_fp64}); mask encrypt {t_mask:.1f} ms, aggregate "
            f"{t_agg:.1f} ms, model decrypt {t_dec_agg:.1f} ms; max |err| vs FP64 mean {max(errs):.2e}")

    if args.stages:
        trip = torch.empty((P, 3, nq, N), dtype=torch.int64, device="cuda")
        t_a2 = event_time(torch, lambda: srv.pair_triples(cts, out=trip))
        del trip
        t_pipe = event_time(torch, lambda: srv.pairwise_sqdist(cts, plan=plan, sumdis=True, out=dist,
                                                               sumdis_out=sumdis))
        t_mask = event_time(torch, lambda: srv.masked_sum(cts, masks, out=agg))
        t_dec = event_time(torch, lambda: kgc.decrypt(dist, out=dec))
        extra["stage_ms"] = {"pair_triples": t_a2, "pairwise_total": t_pipe, "masked_sum": t_mask, "decrypt": t_dec}
        log(f"[bench] stages (ms): {extra['stage_ms']}")

    # ---- plain per-op form on a few pairs (lc_ct_sub / lc_ct_square / lc_ct_add per ciphertext) ------
    if args.per_op_pairs:
        pairs = [(0, 1), (n - 2, n - 1), (0, n - 1)][: args.per_op_pairs]
        tmp = torch.empty((1, 2, nq, N), dtype=torch.int64, device="cuda")
        sq = torch.empty((1, 3, nq, N), dtype=torch.int64, device="cuda")
        acc = torch.empty((1, 3, nq, N), dtype=torch.int64, device="cuda")
        out2 = torch.empty((1, 2, nq, N), dtype=torch.int64, device="cuda")

        def per_op():
            for (i, j) in pairs:
                acc.zero_()
                for k in range(ln):
                    srv.ct_sub(cts[i, k], cts[j, k], out=tmp)
                    srv.ct_square(tmp, out=sq)
                    srv.ct_add(acc, sq, out=acc, ncomp=3)
                srv.relin(acc, out=out2)
                srv.rotate_sum(out2, plan)

        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        per_op()
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        extra["per_op_form"] = {"pairs_timed": len(pairs), "seconds_per_pair": tp / len(pairs),
                                "distances_per_s": len(pairs) / tp}
        log(f"[bench] per-op form: {tp / len(pairs) * 1e3:.1f} ms/pair -> {len(pairs) / tp:.2f} distances/s")

    # ---- ablations of the paper's two techniques (Lazy Relinearization, Dynamic Hoisting) ----------
    if args.ablation:
        ab = {"hoisting_plan_ms": {k: v for k, v in tuned.get("plan_ms", {}).items()}}
        # eager relinearization in the per-op form, one pair: relinearize every
        # square, then add the 2-component results (LEN key switches per pair
        # instead of one)
        i0, j0 = 0, n - 1
        tmp = torch.empty((1, 2, nq, N), dtype=torch.int64, device="cuda")
        sq = torch.empty((1, 3, nq, N), dtype=torch.int64, device="cuda")
        r2 = torch.empty((1, 2, nq, N), dtype=torch.int64, device="cuda")
        acc2 = torch.empty((1, 2, nq, N), dtype=torch.int64, device="cuda")
        acc3 = torch.empty((1, 3, nq, N), dtype=torch.int64, device="cuda")
        out2 = torch.empty((1, 2, nq, N), dtype=torch.int64, device="cuda")

        def eager():
            acc2.zero_()
            for k in range(ln):
                srv.ct_sub(cts[i0, k], cts[j0, k], out=tmp)
                srv.ct_square(tmp, out=sq)
                srv.relin(sq, out=r2)
                srv.ct_add(acc2, r2, out=acc2)
            srv.rotate_sum(acc2, plan)

        def lazy():
            acc3.zero_()
            for k in range(ln):
                srv.ct_sub(cts[i0, k], cts[j0, k], out=tmp)
                srv.ct_square(tmp, out=sq)
                srv.ct_add(acc3, sq, out=acc3, ncomp=3)
            srv.relin(acc3, out=out2)
            srv.rotate_sum(out2, plan)

        t_eager = event_time(torch, eager)
        t_lazy = event_time(torch, lazy)
        d_e = kgc.crt_to_double(kgc.decrypt(acc2)[0, :, :1].cpu().numpy().view(np.uint64))[0] / scale ** 2
        d_l = kgc.crt_to_double(kgc.decrypt(out2)[0, :, :1].cpu().numpy().view(np.uint64))[0] / scale ** 2
        ab["relin_per_op_one_pair"] = {"eager_ms": t_eager, "lazy_ms": t_lazy, "speedup": t_eager / t_lazy,
                                       "key_switches_eager": ln + len(plan), "key_switches_lazy": 1 + len(plan),
                                       "distance_eager": d_e, "distance_lazy": d_l}
        del tmp, sq, r2, acc2, acc3, out2
        # SumDis with one relinearization and rotate-and-sum per client
        # (lc_sumdis_lazy): the triples of all pairs (i, j) are summed per
        # client i first (n key-switch chains instead of P)
        s2 = torch.empty((n, 2, nq, N), dtype=torch.int64, device="cuda")
        t_sd = event_time(torch, lambda: srv.sumdis_lazy(cts, plan=plan, out=s2))
        t_full = extra["stage_ms"]["pairwise_total"] if "stage_ms" in extra else None
        ds = kgc.crt_to_double(kgc.decrypt(s2)[:, :, 0].cpu().numpy().view(np.uint64).T.copy()) / scale ** 2
        dref = kgc.crt_to_double(kgc.decrypt(sumdis)[:, :, 0].cpu().numpy().view(np.uint64).T.copy()) / scale ** 2
        ab["sumdis_per_client_relin"] = {"ms": t_sd, "pairwise_with_sumdis_ms": t_full,
                                        "key_switch_chains": n, "vs_pairwise_chains": P,
                                        "max_rel_diff_vs_pairwise_sumdis": float(np.max(np.abs(ds - dref) / np.abs(dref)))}
        del s2
        extra["ablation"] = ab
        log(f"[bench] ablation: eager relin {t_eager:.0f} ms vs lazy {t_lazy:.0f} ms per pair "
            f"({t_eager / t_lazy:.1f}x); SumDis with per-client relin {t_sd:.0f} ms "
            f"(max rel diff {ab['sumdis_per_client_relin']['max_rel_diff_vs_pairwise_sumdis']:.1e})")

    # ---- roofline of the dominant kernel ------------------------------------------
    # Candidates: the fused pair-triple kernel (one launch per step, FP64-ALU
    # bound: 23 FP64 lane-instructions per update in the Barrett form -- two
    # subtractions, three products of six instructions, three accumulations)
    # and the NTT passes of the key switches (HBM bound; the figure is one
    # forward transform of 64 ciphertexts' limbs, timed, over its two
    # launches, and its share of the step is that time per limb-transform
    # times the limb-transforms a step performs).  The `roofline` entry is
    # the candidate with the larger estimated share of the step.
    roof = None
    if args.stages:
        nt = ntt_roofline(torch, srv, 64 if w.log_n >= 15 else 256)
        ks_count = P * (1 + len(plan))
        limb_ntts_per_ks = nq + srv.dnum * nq + 2 * srv.np + 2 * nq  # (L+1+K-alpha) = L+1 as alpha = K
        ntt_ms_step = ks_count * limb_ntts_per_ks * nt["transform_ms_per_limb_poly"]
        updates = P * ln * nq * N
        a2_bytes = n * ln * 2 * nq * N * 8 + P * 3 * nq * N * 8
        if tuned.get("pair_mfma"):  # the Gram form: HBM-bound by design (ciphertexts read once)
            a2 = {"bound": "hbm", "achieved": a2_bytes / (extra["stage_ms"]["pair_triples"] / 1e3) / 1e9,
                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": None, "kernel": "pair_gram_kernel",
                  "units_per_launch": "%d bytes of ciphertexts in and triples out" % a2_bytes,
                  "launch_ms": extra["stage_ms"]["pair_triples"], "est_ms_per_step": extra["stage_ms"]["pair_triples"]}
        else:
            a2 = {"bound": "alu",
                  "achieved": A2_OPS_PER_UPDATE * updates / (extra["stage_ms"]["pair_triples"] / 1e3) / 1e12,
                  "peak": VALU_PEAK_TOPS, "unit": "T FP64 lane-ops/s", "traffic": None, "kernel": "pair_triples_kernel",
                  "units_per_launch": "%d updates x %d FP64 lane-ops" % (updates, A2_OPS_PER_UPDATE),
                  "launch_ms": extra["stage_ms"]["pair_triples"], "est_ms_per_step": extra["stage_ms"]["pair_triples"]}
        ntt = {"bound": "hbm", "achieved": nt["bytes_per_launch"] / (nt["launch_ms"] / 1e3) / 1e9,
               "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": None, "kernel": "ntt_fast_kernel",
               "units_per_launch": "%d limb-polys x 8N bytes (16N per transform over its two launches)"
                                   % nt["limb_polys"],
               "launch_ms": nt["launch_ms"], "est_ms_per_step": ntt_ms_step}
        for r in (a2, ntt):
            r["frac"] = r["achieved"] / r["peak"]
        if not tuned.get("pair_mfma") and A2_PMC["source_sha256"] == _source_sha256(*A2_SECTION):
            a2["traffic"] = A2_PMC["fetch_bytes"] + A2_PMC["write_bytes"]
            a2["traffic_vs_algorithmic"] = a2["traffic"] / a2_bytes
        if NTT_PMC and NTT_PMC["source_sha256"] == _source_sha256(*NTT_SECTION) and nt["limb_polys"] == NTT_PMC["limb_polys"]:
            ntt["traffic"] = NTT_PMC["fetch_bytes_per_launch"] + NTT_PMC["write_bytes_per_launch"]
            ntt["traffic_vs_algorithmic"] = ntt["traffic"] / nt["bytes_per_launch"]
            ntt["traffic_GBps"] = ntt["traffic"] / (nt["launch_ms"] / 1e3) / 1e9
        roof = max((a2, ntt), key=lambda r: r["est_ms_per_step"])
        extra["kernels"] = {"pair_triples": a2, "ntt": ntt, "reported": roof["kernel"]}
        log(f"[bench] a2 kernel {a2['launch_ms']:.1f} ms ({a2['achieved']:.2f} T FP64 ops/s, {a2['frac']:.1%} of VALU); "
            f"NTT {ntt['achieved']:.0f} GB/s per launch ({ntt['frac']:.1%} of HBM), ~{ntt_ms_step:.0f} ms/step; "
            f"reported: {roof['kernel']}")

    # the round's ciphertexts are no longer needed
    used_graph = graph is not None
    del cts, dist, sumdis, agg, dec, masks, graph
    torch.cuda.synchronize()
    for ctx_ in (srv, kgc):  # the graph is gone: give back the timed stream's workspaces
        ctx_.release_workspace()
    torch.cuda.empty_cache()

    if args.ntt_micro:
        extra["ntt_micro"] = ntt_micro(torch, L)
        torch.cuda.empty_cache()

    if args.sweep_n:
        extra["n_sweep"] = sweep_n(torch, L, synth)
        torch.cuda.empty_cache()

    if args.serve:
        if w.log_n != 16:
            log("[bench] --serve needs the N=2^16 workload's contexts; skipped")
        else:
            extra["serving"] = serve_bench(args, torch, L, srv, kgc, plan)

    small_plans = []
    if args.small_configs and w.log_n == 16:
        extra["configs"] = {}
        for sw in (synth.CFG1, synth.CFG2):
            extra["configs"][sw.name] = small_config(torch, L, synth, sw)
            small_plans.append((sw, extra["configs"][sw.name]["batched"]["plan"]))
            torch.cuda.empty_cache()

    base = None
    if args.cpu_baseline:
        log("[bench] timing the CPU oracle: one whole pair of this workload, the smaller workloads in full")
        base = cpu_baseline(w, plan, small_plans)
        log(f"[bench] oracle: {base['value']:.4f} distances/s ({base['sample']}); one thread "
            f"{base['one_thread']['seconds']} s vs {base['one_thread']['seconds_all_threads']:.2f} s on "
            f"{base['cores']} threads ({base['cpu']['model']})")

    out = {
        "metric": "encrypted client-pair distances/s at N=2^16",
        "value": value,
        "unit": "client-pair distances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w.name, "N": N, "limbs": nq, "special_primes": srv.np, "dnum": srv.dnum,
                   "clients": n, "dim": w.dim, "ciphertexts_per_client": ln, "pairs": P, "plan": plan,
                   "scale_log2": w.scale_log2},
        "check": check,
        "hip_graph": used_graph,
        "ingest_s": {"h2d": t_h2d, "encode_device": t_enc_dev, "encrypt_device": t_encrypt, "keygen": t_keys,
                     **host_cmp},
        "roofline": roof,
        "cpu_baseline": base,
    }
    out["autotune"] = tuned
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
