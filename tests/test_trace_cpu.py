"""roctx ranges: off by default, on when RX_ROCTX is set and a roctx library can be opened; compiling and
the other host paths behave the same either way."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = ("from paper_1108_3126_amd import rx; p = rx.compile_regex(b'a(b|c)*d', search=True); "
         "print(rx.lib().rx_trace_enabled(), p.info.m)")


def run(env_extra):
    env = dict(os.environ)
    env.pop("RX_ROCTX", None)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", PROBE], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stdout.split()


def test_ranges_off_by_default():
    assert run({}) == ["0", "14"]
    assert run({"RX_ROCTX": "0"}) == ["0", "14"]


def test_ranges_on_with_rx_roctx():
    have = any(os.path.exists(os.path.join("/opt/rocm/lib", n))
               for n in ("librocprofiler-sdk-roctx.so.1", "libroctx64.so.4"))
    assert run({"RX_ROCTX": "1"}) == ["1" if have else "0", "14"]
