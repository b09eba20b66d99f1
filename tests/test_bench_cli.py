"""bench.py's command line, checked without a GPU: more than one GPU is refused with a
message before anything touches a device, and --help lists the single-workload flag."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and "requested 2" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_help_lists_single_workload_flag():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--only", "--no-cpu-baseline"):
        assert flag in r.stdout


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_file_matches_kernel_source_and_is_consistent():
    # the committed Gram counter summary was taken on the current kernel source, so the bench
    # reports its traffic; its figures agree with each other and with a physical lower bound
    b = _bench_module()
    vals = {}
    with open(b.COUNTERS_FILE) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.split("#")[0].strip()
    assert vals["kernel_source_sha256_16"] == b._src_hash("ncc.hip", "queue.hpp")
    rd, wr = float(vals["hbm_read_bytes_per_launch"]), float(vals["hbm_write_bytes_per_launch"])
    assert abs(float(vals["fetch_scale"]) - 1048576 / float(vals["copy_fetch_size_kib"])) <= 1e-5
    assert abs(rd - float(vals["fetch_size_kib"]) * 1024 * float(vals["fetch_scale"])) <= 1e-5 * rd
    assert abs(wr - float(vals["write_size_kib"]) * 1024) <= 1e-5 * wr
    total = b._traffic_from_profile()
    assert total is not None and abs(total - (rd + wr)) <= 1e-5 * total
    n, d = 4096, 1 << 20
    assert rd >= n * d * 3 * 2          # every prepared bf16 operand plane is read at least once
    assert wr >= n * (n - 1) // 2 * 4   # every pair's f32 result is written


def test_traffic_is_dropped_when_the_kernel_source_changes(monkeypatch):
    b = _bench_module()
    monkeypatch.setattr(b, "_src_hash", lambda *names: "0000000000000000")
    assert b._traffic_from_profile() is None


def test_profile_commands_use_existing_bench_flags():
    # every rocprofv3 command recorded in profiles/ runs bench.py with flags it accepts
    import glob
    import re
    helptext = _run("--help").stdout
    cmds = []
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.txt")):
        with open(path) as f:
            for line in f:
                if line.startswith("#") and "rocprofv3" in line and "bench.py" in line:
                    assert "-- python3 bench.py" in line, line  # the program runs directly after --
                    cmds.append((os.path.basename(path), line.split("bench.py", 1)[1]))
    assert len(cmds) >= 8
    for name, args in cmds:
        for flag in re.findall(r"--[a-z][a-z0-9-]*", args):
            assert flag in helptext, (name, flag)
        m = re.search(r"--only (\S+)", args)
        if m:
            assert m.group(1) in ("clouds", "sparse", "cv", "pce", "pce_big", "pce_camera", "ooc", "small", "valu",
                                  "forensics"), (name, m.group(1))
