"""bench.py on the CPU: a request for more than one GPU stops with a message,
before anything touches a device; counter-measured traffic is reported only
for the kernel sources it was measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_measured_traffic_is_reported_only_for_the_sources_it_was_measured_on(monkeypatch):
    """roofline.traffic comes from counter runs of one version of the kernel
    sources: for any other version (another hash) it is null, and workloads
    that were never measured are null too."""
    bench = _bench_module()
    key = "cube1024_persp1920x1080/f32/composite/fixed"
    stored = bench.MEASURED_TRAFFIC["bytes"][key]
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "sources_sha256", bench.kernel_sha256())
    assert bench.measured_traffic(key) == stored
    assert bench.measured_traffic("cube128_ortho256/f32/composite/fixed") is None
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "sources_sha256", "0" * 64)
    assert bench.measured_traffic(key) is None
    # every stored figure is a byte count of a workload bench.py knows
    for k, v in bench.MEASURED_TRAFFIC["bytes"].items():
        workload, storage, op, step = k.split("/")
        assert workload in bench.WORKLOADS and storage in ("f32", "f16", "fp8")
        assert op in ("composite", "mip") and step in ("fixed", "voxel")
        assert isinstance(v, int) and v > 0


def test_kernel_hash_covers_every_ray_caster_source():
    bench = _bench_module()
    csrc = os.path.join(ROOT, "paper_1205_0282_amd", "csrc")
    for name in bench.KERNEL_SOURCES:
        assert os.path.isfile(os.path.join(csrc, name)), name
    # the sources the ray caster is compiled from (its own file and every
    # local header it includes, directly or not) are all hashed
    seen, todo = set(), ["bc_render.hip"]
    while todo:
        name = todo.pop()
        if name in seen:
            continue
        seen.add(name)
        with open(os.path.join(csrc, name)) as fh:
            todo += [ln.split('"')[1] for ln in fh if ln.startswith("#include \"")]
    assert seen <= set(bench.KERNEL_SOURCES)
