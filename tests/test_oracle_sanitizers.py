"""The CPU oracle under the host sanitizers: every entry point on a tiny nested
grid, built with AddressSanitizer + UndefinedBehaviorSanitizer (sequential and
threaded transport) and with ThreadSanitizer (threaded transport)."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "oracle_sanitize_main.c"), os.path.join(HERE, "..", "oracle", "mcrt_oracle.c")]


def _build_and_run(tmp_path, flags, threads, sources=SRC):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    exe = str(tmp_path / "drv")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", *flags, "-o", exe, *sources, "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "sanitizer" in b.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + b.stderr[-200:])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="report_signal_unsafe=0", OMP_NUM_THREADS=str(threads))
    r = subprocess.run([exe, str(threads)], capture_output=True, text=True, env=env, timeout=300)
    return r


@pytest.mark.parametrize("threads", [1, 4])
def test_oracle_clean_under_asan_ubsan(tmp_path, threads):
    r = _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"], threads)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.startswith("ok ")


_ACCESS = re.compile(r"^  (?:Previous )?(?:atomic )?(?:read|write|Read|Write) of size \d+ at \S+ by .*:$")


def _races_between_workers(stderr):
    """ThreadSanitizer reports whose two accesses both sit inside the same
    parallel region.  libgomp is not instrumented, so its fork and join are invisible to
    the sanitizer and it reports the code before and after a region (the
    region's argument block on the caller's stack, the results read after the
    join, a later region reading them) against the workers; those reports are
    dropped here."""
    real = []
    for rep in stderr.split("WARNING: ThreadSanitizer")[1:]:
        lines = rep.split("\n")
        stacks = []
        for k, line in enumerate(lines):
            if _ACCESS.match(line):
                st = []
                for q in lines[k + 1:]:
                    if not q.strip():
                        break
                    st.append(q)
                stacks.append("\n".join(st))
        regions = [set(re.findall(r"\S+\._omp_fn\.\d+", st)) for st in stacks[:2]]
        if len(regions) == 2 and regions[0] & regions[1]:
            real.append(rep)
    return real


def test_oracle_threaded_transport_clean_under_tsan(tmp_path):
    r = _build_and_run(tmp_path, ["-fsanitize=thread"], 4)
    if "FATAL: ThreadSanitizer" in r.stderr and "unexpected memory mapping" in r.stderr:
        pytest.skip("ThreadSanitizer cannot map its shadow memory in this environment")
    real = _races_between_workers(r.stderr)
    assert not real, real[0]
    if "WARNING: ThreadSanitizer" not in r.stderr:
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.startswith("ok ")


def test_tsan_filter_catches_a_planted_race(tmp_path):
    """The report filter above keeps a real race: a copy of the oracle whose
    shared counters are updated without atomics must be reported."""
    src = open(SRC[1]).read()
    atomic = "if (threaded) return __atomic_fetch_add(a, v, __ATOMIC_RELAXED);"
    assert atomic in src
    (tmp_path / "oracle").mkdir()
    (tmp_path / "tests").mkdir()
    (tmp_path / "oracle" / "mcrt_oracle.c").write_text(src.replace(atomic, "(void)threaded;"))
    shutil.copy(os.path.join(HERE, "..", "oracle", "mcrt_oracle.h"), tmp_path / "oracle")
    shutil.copy(SRC[0], tmp_path / "tests")
    planted = [str(tmp_path / "tests" / "oracle_sanitize_main.c"), str(tmp_path / "oracle" / "mcrt_oracle.c")]
    r = _build_and_run(tmp_path, ["-fsanitize=thread"], 4, planted)
    if "FATAL: ThreadSanitizer" in r.stderr and "unexpected memory mapping" in r.stderr:
        pytest.skip("ThreadSanitizer cannot map its shadow memory in this environment")
    assert _races_between_workers(r.stderr)
