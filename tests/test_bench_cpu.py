"""Host logic of bench.py: the source fingerprint that ties the committed HBM-traffic profile
to the kernel it was taken on."""
import importlib.util
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    sys.modules["bench_mod"] = mod          # its worker functions pickle by module name
    spec.loader.exec_module(mod)
    return mod


def test_code_sha256_ignores_comments_and_blank_lines(tmp_path):
    b = _bench()
    base = "int f(int x) {\n  return x + 1;\n}\n"
    commented = "// header\nint f(int x) {   // trailing note\n\n  return x + 1;  \n}\n\n"
    changed = "int f(int x) {\n  return x + 2;\n}\n"
    paths = []
    for k, text in enumerate((base, commented, changed)):
        p = tmp_path / f"k{k}.hip"
        p.write_text(text)
        paths.append(str(p))
    h = [b.code_sha256(p) for p in paths]
    assert h[0] == h[1]
    assert h[0] != h[2]


def test_profiled_traffic_is_none_for_an_unknown_source(tmp_path, monkeypatch):
    b = _bench()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "t.json").write_text('{"fine_hip_code_sha256": "0", "fetch_bytes_per_launch": 1e9, '
                                 '"write_bytes_per_launch": 1e9}')
    csrc = tmp_path / "paper_2510_26180_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("int x;\n")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.profiled_traffic("k.hip", "t.json") is None
    (prof / "t.json").write_text('{"fine_hip_code_sha256": "%s", "fetch_bytes_per_launch": 1e9, '
                                 '"write_bytes_per_launch": 2e9}' % b.code_sha256(str(csrc / "k.hip")))
    assert b.profiled_traffic("k.hip", "t.json") == 3.0


def test_profiled_traffic_is_none_for_another_launch_shape(tmp_path, monkeypatch):
    b = _bench()
    prof = tmp_path / "profiles"
    prof.mkdir()
    csrc = tmp_path / "paper_2510_26180_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("int x;\n")
    shape = {"n": 128, "N": 64, "J": 64, "M": 256, "variant": 6, "launches": 16}
    import json
    (prof / "t.json").write_text(json.dumps({"fine_hip_code_sha256": b.code_sha256(str(csrc / "k.hip")),
                                             "fetch_bytes_per_launch": 1e9, "write_bytes_per_launch": 2e9,
                                             "shape": shape}))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.profiled_traffic("k.hip", "t.json", dict(shape)) == 3.0
    assert b.profiled_traffic("k.hip", "t.json", dict(shape, M=512)) is None
    assert b.profiled_traffic("k.hip", "t.json", dict(shape, variant=5)) is None


def test_cpu_leg_serial_fine_and_baseline():
    """The oracle leg on a small 2D problem with two forked workers: the serial fine solutions
    of the subset are the oracle's, and the baseline names its worker count."""
    import multiprocessing as mp

    import numpy as np

    import workloads as W
    from oracle import field, prop
    b = _bench()
    w = W.small_2d(n=8, N=4, J=2)
    xi = W.draw_xi(4, w.d, 5)
    pool = mp.get_context("fork").Pool(2, initializer=b._oracle_init)
    try:
        base, refs = b.cpu_baseline(pool, 2, w, xi, [0, 3], 4.0)
    finally:
        pool.close()
        pool.join()
    assert base["cores"] == 2 and base["kind"] == "oracle" and base["value"] > 0
    lam, Phi = field.kl_modes(w.dim, w.n, w.d, w.corr_len, w.sigma)
    for j, m in enumerate([0, 3]):
        a = field.synthesize(lam, Phi, xi[m:m + 1])[0]
        want = prop.serial_fine(prop.Propagators(w.dim, w.n, a, w.T, w.N, w.J, w.forcing), np.zeros(w.Nx), w.N)
        assert np.array_equal(refs[j], want)


def test_subset_draw_is_seeded_and_distinct():
    import numpy as np

    import workloads as W
    s = W.draw_subset(256, 16, 2009)
    assert len(set(s.tolist())) == 16 and np.all(np.diff(s) > 0) and s.max() < 256
    assert np.array_equal(s, W.draw_subset(256, 16, 2009))


def test_profile_summaries_run_committed_files_only():
    # every summary under profiles/ is short text whose commands run files of the repository
    import re
    import subprocess
    tracked = set(subprocess.run(["git", "ls-files"], cwd=ROOT, capture_output=True, text=True,
                                 check=True).stdout.split())
    pdir = os.path.join(ROOT, "profiles")
    names = sorted(os.listdir(pdir))
    assert names
    for name in names:
        path = os.path.join(pdir, name)
        assert name.endswith((".md", ".txt", ".json")), name
        assert os.path.getsize(path) < 64 * 1024, name
        text = open(path).read()
        assert "_work/" not in text and "gpurun" not in text, name
        if name.endswith(".md"):
            assert "rocprofv3" in text or "python" in text, name
            for script in re.findall(r"python3?\s+(?:-u\s+)?([\w/.-]+\.py)", text):
                assert script in tracked, (name, script)
