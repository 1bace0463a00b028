"""Host logic of bench.py: the source fingerprint that ties the committed HBM-traffic profile
to the kernel it was taken on."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
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
