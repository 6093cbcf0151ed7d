"""The reconstruction service on the GPU: results are the same alone and in
the mix (bitwise: every request has its own plan and fixed-order
reductions), and a mixed trace completes under continuous batching."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_results_identical_alone_and_in_the_mix():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_11511_amd import lib
    from paper_2008_11511_amd.serve import serve_trace
    lib()
    kw = dict(n_requests=6, rate=40.0, seed=5, sizes=(64, 128), min_frames=60, max_frames=160,
              schedule=(("dm", 4), ("ml", 3)), min_side=256)
    say("serve: continuous")
    con, s_con = serve_trace(max_active=6, **kw)
    say("serve: sequential")
    seq, s_seq = serve_trace(sequential=True, **kw)
    assert s_con["requests"] == s_seq["requests"] == 6
    for a, b in zip(con, seq):
        assert a.rid == b.rid
        assert np.array_equal(a.result["obj"], b.result["obj"])
        assert np.array_equal(a.result["probe"], b.result["probe"])
        assert a.result["llk"] == b.result["llk"]
        assert np.isfinite(a.result["llk"])


def test_results_identical_when_requests_run_concurrently():
    """Two running lanes (the oldest request and the shortest other one) put
    two requests' cycles on the device at once; every result is still bitwise
    its sequential run."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_11511_amd import lib
    from paper_2008_11511_amd.serve import serve_trace
    lib()
    kw = dict(n_requests=8, rate=60.0, seed=9, sizes=(64, 128, 256), min_frames=60, max_frames=200,
              schedule=(("dm", 6), ("ml", 4)), min_side=320)
    say("serve: two concurrent lanes")
    con, s_con = serve_trace(max_active=8, max_running=2, order="lanes", **kw)
    say("serve: sequential")
    seq, s_seq = serve_trace(sequential=True, **kw)
    assert s_con["max_requests_in_flight"] >= 2          # two requests' work was queued on the device at once
    assert s_seq["max_requests_in_flight"] == 1
    assert len({(r.wl.n, r.wl.n_modes) for r in con}) >= 3
    for a, b in zip(con, seq):
        assert a.rid == b.rid
        assert np.array_equal(a.result["obj"], b.result["obj"])
        assert np.array_equal(a.result["probe"], b.result["probe"])
        assert np.array_equal(a.result["llk_history"], b.result["llk_history"])


def _scan(seed, n, k, j, side, mask_frac):
    """A small caller-side reconstruction problem: data from the oracle's
    forward model and a Poisson draw, starts as in the benchmarks."""
    import oracle
    import synth
    obj = synth.object_truth((side, side), seed)
    probe = synth.probe_modes(n, k, seed)
    offs = oracle.offsets_from_positions(synth.spiral_positions(j, n / 10.0), n, (side, side))
    probe = probe * synth.probe_photon_scale(obj, probe, offs, 1e6)
    iobs = synth.poisson_counts(oracle.simulate_intensity(obj, probe, offs), seed).astype(np.float32)
    mask = synth.gap_mask(n, mask_frac, seed)
    obj0 = synth.perturb_object(obj, seed).astype(np.complex64)
    probe0 = synth.perturb_probe(probe, seed).astype(np.complex64)
    return dict(iobs=iobs, offsets=offs.astype(np.int32), obj0=obj0, probe0=probe0, mask=mask)


SCHED = (("dm", 4), ("ml", 3))


def _direct(sc, dev):
    """The same schedule run directly on a plan."""
    from paper_2008_11511_amd import Plan
    iobs = torch.from_numpy(sc["iobs"]).to(dev)
    mask = torch.from_numpy(sc["mask"]).to(dev) if sc["mask"] is not None else None
    o = torch.from_numpy(sc["obj0"]).to(dev)
    p = torch.from_numpy(sc["probe0"]).to(dev)
    plan = Plan(sc["offsets"], iobs, mask, p.shape[0], tuple(o.shape))
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 4, 3)
    st = plan.ml_state()
    hist = torch.zeros(3, dtype=torch.float64, device=dev)
    plan.ml_cycle(o, p, st, 3, 3, reset=True, hist=hist)
    llk = plan.llk(o, p)
    torch.cuda.synchronize()
    l = llk.cpu().numpy()
    return o.cpu().numpy(), p.cpu().numpy(), l[0] / l[1], hist.cpu().numpy() / l[1]


def test_service_results_equal_direct_runs_and_a_low_budget_queues_requests():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_11511_amd import lib
    from paper_2008_11511_amd.serve import ReconstructionService
    lib()
    dev = torch.device("cuda:0")
    say("service: three caller-supplied scans")
    scans = [_scan(31, 64, 1, 80, 256, 0.0), _scan(32, 128, 2, 60, 384, 0.03), _scan(33, 64, 3, 100, 288, 0.03)]
    ref = [_direct(sc, dev) for sc in scans]
    for budget in (None, "low"):
        kw = {}
        if budget == "low":
            # room for one request at a time: the others wait for memory
            from paper_2008_11511_amd.serve import GpuExecutor, Request, Scan
            need = max(GpuExecutor.footprint(Request(0, 0.0, Scan(s["iobs"].shape[1], s["probe0"].shape[0],
                                                                  s["iobs"].shape[0], s["obj0"].shape),
                                                     SCHED, data={})) for s in scans)
            kw = dict(hbm_budget=int(need * 1.3))
        say(f"service: budget {budget}")
        with ReconstructionService(**kw) as svc:
            futs = []
            for i, sc in enumerate(scans):
                args = dict(sc)
                if i == 1:             # device inputs are accepted too
                    args["iobs"] = torch.from_numpy(sc["iobs"]).to(dev)
                futs.append(svc.submit(schedule=SCHED, **args))
            res = [f.result(timeout=120) for f in futs]
            if budget == "low":
                admits = [e for e in svc.sch.log if e[0] == "admit"]
                assert max(e[3] for e in admits) <= int(need * 1.3)
        for r, (o, p, llk, hist) in zip(res, ref):
            assert np.array_equal(r["obj"], o)
            assert np.array_equal(r["probe"], p)
            assert r["llk"] == llk
            np.testing.assert_array_equal(r["llk_history"], hist)
            assert r["timings"]["latency_s"] >= r["timings"]["service_s"] > 0


def test_service_refuses_a_scan_outside_the_object():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_11511_amd import PtychoError, lib
    from paper_2008_11511_amd.serve import ReconstructionService
    lib()
    sc = _scan(34, 64, 1, 20, 256, 0.0)
    sc["offsets"] = sc["offsets"].copy()
    sc["offsets"][5] = (250, 0)                    # window leaves the 256 x 256 object
    with ReconstructionService() as svc:
        with pytest.raises(PtychoError) as e:
            svc.submit(schedule=SCHED, **sc)
        assert e.value.code == -2


def test_service_fails_a_diverging_request_and_serves_the_others():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_11511_amd import lib
    from paper_2008_11511_amd.serve import ReconstructionService
    lib()
    say("service: one request with NaN data among good ones")
    scans = [_scan(41, 64, 1, 40, 256, 0.0), _scan(42, 64, 2, 40, 256, 0.03), _scan(43, 64, 1, 40, 256, 0.0)]
    scans[1]["iobs"] = scans[1]["iobs"].copy()
    scans[1]["iobs"][3, 10, 10] = np.nan
    with ReconstructionService() as svc:
        futs = [svc.submit(schedule=SCHED, **sc) for sc in scans]
        with pytest.raises(FloatingPointError):
            futs[1].result(timeout=120)
        good = [futs[0].result(timeout=120), futs[2].result(timeout=120)]
    for r in good:
        assert np.isfinite(r["obj"]).all() and np.isfinite(r["llk"])


def test_service_serves_near_field_and_far_field_scans_together():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import synth
    from paper_2008_11511_amd import Plan, lib
    from paper_2008_11511_amd.serve import ReconstructionService
    lib()
    dev = torch.device("cuda:0")
    say("service: a near-field scan beside a far-field one")
    n, side, seed = 64, 160, 41
    f = synth.fresnel_parameter(n, 0.02)
    obj = synth.object_truth((side, side), seed)
    probe = synth.near_field_probe(n, 1, seed)
    offs = oracle.offsets_from_positions(synth.random_positions(20, 64.0, seed), n, (side, side))
    probe = probe * synth.probe_photon_scale(obj, probe, offs, 1e4 * n * n)
    near = dict(iobs=synth.poisson_counts(oracle.simulate_intensity(obj, probe, offs, nf=f), seed).astype(np.float32),
                offsets=offs.astype(np.int32), obj0=synth.start_object((side, side)).astype(np.complex64),
                probe0=synth.start_probe(probe).astype(np.complex64), mask=None)
    far = _scan(42, 64, 2, 60, 256, 0.03)
    # the near-field reference, run directly
    o = torch.from_numpy(near["obj0"]).to(dev)
    p = torch.from_numpy(near["probe0"]).to(dev)
    plan = Plan(near["offsets"], torch.from_numpy(near["iobs"]).to(dev), None, 1, (side, side), near_field=f)
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 4, 3)
    st = plan.ml_state()
    plan.ml_cycle(o, p, st, 3, 3, reset=True)
    ref_o = o.cpu().numpy()
    ref_far = _direct(far, dev)
    with ReconstructionService() as svc:
        fn = svc.submit(schedule=SCHED, near_field=f, **near)
        ff = svc.submit(schedule=SCHED, **far)
        rn, rf = fn.result(timeout=120), ff.result(timeout=120)
    assert np.array_equal(rn["obj"], ref_o)
    assert np.array_equal(rf["obj"], ref_far[0])
    with ReconstructionService() as svc2:
        with pytest.raises(ValueError, match="finite"):
            svc2.submit(schedule=SCHED, near_field=float("nan"), **near)


def test_synthetic_near_field_request_in_a_trace():
    """A synthetic near-field request (data drawn on the device from the
    near-field forward model) beside far-field ones: the same result in the
    continuous and the sequential schedule."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import dataclasses
    import synth
    from paper_2008_11511_amd import lib
    from paper_2008_11511_amd.serve import GpuExecutor, Request, Scheduler, make_trace
    lib()
    nf = dataclasses.replace(synth.workload("nf1024"), name="nf64", n=64, n_frames=20, obj_shape=(160, 160),
                             step=64.0, photons=1e4 * 64 * 64, fresnel=synth.fresnel_parameter(64, 0.02))

    def run(sequential):
        reqs = make_trace(3, 40.0, 5, sizes=(64,), min_frames=60, max_frames=100, schedule=SCHED, min_side=256)
        reqs.append(Request(3, 0.02, nf, SCHED))
        ex = GpuExecutor("cuda:0")
        for r in reqs:
            ex.prepare(r)
        free, _ = torch.cuda.mem_get_info(torch.device("cuda:0"))
        budget = int(0.5 * free)
        ex.attach_arena(int(budget * 0.85))
        Scheduler(ex, budget, max_active=6, sequential=sequential).run(reqs)
        ex.close()
        return reqs

    say("serve: synthetic near-field request, continuous")
    con = run(False)
    say("serve: synthetic near-field request, sequential")
    seq = run(True)
    for a, b in zip(con, seq):
        assert a.error is None and b.error is None
        assert np.array_equal(a.result["obj"], b.result["obj"])
        assert a.result["llk"] == b.result["llk"] and np.isfinite(a.result["llk"])
    # the near-field request fits its own data: the final LLK per pixel is a
    # few units (Poisson noise), not the far-field model's mismatch
    assert con[3].result["llk"] < 50.0
