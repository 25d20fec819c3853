"""Host-side set-up of the serving path (no GPU): the projector table a
request builds on host threads, in chunks of k-points, equals the plain
per-k construction (every plane wave of every k in the library's order,
zero padding)."""
import numpy as np

from paper_2412_01695_amd import mkpw, serve, synth


def test_projector_table_matches_per_k_construction():
    reqs = [r for r in serve.make_requests(40, 20.0) if r.cfg.nproj == 8][:2]
    reqs += [r for r in serve.make_requests(40, 20.0) if r.cfg.nproj == 4][:1]
    assert len(reqs) == 3
    for r in reqs:
        cfg = r.cfg
        ctx = mkpw.pw_create(-1, None)
        try:
            mkpw.pw_set_lattice(ctx, cfg.lat)
            mkpw.pw_set_cutoff(ctx, cfg.ecut_ry, cfg.fft)
            npw, npwx = mkpw.pw_set_kpoints(ctx, cfg.kpts)
            mall = mkpw.pw_get_miller_all(ctx, npw)
            got = serve.projector_table(cfg, npw, npwx, mall, kchunk=7)
            ref = np.zeros_like(got)
            for ik in range(cfg.nk):
                m = mkpw.pw_get_miller(ctx, ik, int(npw[ik]))
                ref[ik, :, :npw[ik]] = synth.beta_values(cfg, synth.q_vectors(cfg, ik, m))
            # the same arithmetic per plane wave; only the matrix product's
            # blocking may differ with the chunk size
            assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))
            assert np.all(got[:, :, npwx - 1][np.asarray(npw) < npwx] == 0)
        finally:
            mkpw.pw_destroy(ctx)


def test_bench_serving_sample_reports_instead_of_raising():
    """The bench runs the serving stream in a server process of its own: a
    server that cannot run (here: no GPU) comes back as an error entry, and a
    server that can comes back with its latency summary; neither raises."""
    import bench

    out = bench.serving_sample(2, timeout_s=300)
    assert isinstance(out, dict)
    assert ("error" in out and "command" in out) or ("p50_s" in out and out["requests"] == 2)
