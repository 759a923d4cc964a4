"""Host logic of bench.py: the one-GPU contract and the key that ties a
committed counter summary to the kernel code it was taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_code_key_ignores_comments_but_not_code(tmp_path):
    src = "int f(int a)\n{\n    return a + 1;  // one more\n}\n"
    a = tmp_path / "a.h"
    a.write_text(src)
    b = tmp_path / "b.h"
    b.write_text("/* a block\n   comment */\n" + src.replace("// one more", "// next value") + "\n\n")
    c = tmp_path / "c.h"
    c.write_text(src.replace("a + 1", "a + 2"))
    assert bench.code_text(str(a)) == bench.code_text(str(b))
    assert bench.code_text(str(a)) != bench.code_text(str(c))
    assert "one more" not in bench.code_text(str(a))


def test_counter_summary_key_format():
    """The committed summary carries a key and a byte count per physics in the
    form bench.py parses (whether the key still matches the code is reported
    by the bench as a null traffic field, not asserted here)."""
    import re

    text = open(bench.PHYS_COUNTERS).read()
    kv = dict(re.findall(r"^- (\w+): `?([^`\n]+)`?$", text, re.M))
    for which in ("tti", "elastic"):
        assert re.fullmatch(r"[0-9a-f]{16}", kv[f"{which}_sha"])
        assert float(kv[f"{which}_hbm_bytes_per_step"]) > 0
