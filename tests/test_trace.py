"""Optional roctx markers of the binding (LBW_ROCTX=1): off by default; when
enabled, ROCm's marker library loads and ranges nest. No GPU needed."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_marker_off_by_default():
    from paper_2309_04872_amd import trace

    if os.environ.get("LBW_ROCTX") != "1":
        assert not trace.ENABLED
        with trace.marker("unused"):
            pass
        assert trace._LIB is None


def test_marker_enabled():
    code = ("from paper_2309_04872_amd import trace\n"
            "assert trace.ENABLED\n"
            "with trace.marker('outer'):\n"
            "    with trace.marker('inner'):\n"
            "        pass\n"
            "assert trace._LIB is not None\n"
            "print('ok')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120, cwd=ROOT,
                       env=dict(os.environ, LBW_ROCTX="1"))
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().endswith("ok")
