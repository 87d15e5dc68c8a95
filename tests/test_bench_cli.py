"""bench.py's contract on the host: one GPU only, and the stored traffic figure ties to the committed
counter summary (same kernel sources, same plan, same bytes)."""

import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_figure_matches_the_counter_summary():
    import bench
    text = open(os.path.join(ROOT, "profiles", "k_event_pass_tiled_prod400_pmc.md")).read()
    assert bench.MEASURED_TRAFFIC, "no stored traffic figure"
    for key, nbytes in bench.MEASURED_TRAFFIC.items():
        src, plan = key.split(":")
        assert f"sha256 prefix `{src}`" in text
        assert re.search(rf"\(plan {plan} from the plan table", text)
        assert f"({nbytes} bytes:" in text


def test_source_hash_ignores_comments(tmp_path):
    """The traffic figure follows the kernel code: a comment or blank line does not change the hash,
    a code change does."""
    import shutil
    import bench
    src = os.path.join(ROOT, "paper_1502_07478_amd", "csrc")
    dst = tmp_path / "paper_1502_07478_amd" / "csrc"
    shutil.copytree(src, dst)
    root0 = bench.ROOT
    try:
        bench.ROOT = str(tmp_path)
        h0 = bench.kernel_source_hash()
        f = dst / "jpet_pass.hip"
        text = f.read_text()
        f.write_text("// a comment\n\n" + text.replace("namespace jpet {", "namespace jpet {  /* note */", 1))
        assert bench.kernel_source_hash() == h0
        f.write_text(text + "\nstatic int unused_probe = 0;\n")
        assert bench.kernel_source_hash() != h0
    finally:
        bench.ROOT = root0
