"""The committed rocprofv3 summaries: each names the command that made it, the commands run
committed files only, and every counter summary was taken from the kernel sources as they are
now (its source hash matches), so the roofline figures that quote it describe these kernels."""
import glob
import os

import pytest

from paper_2403_12820_amd import profile_summary as PS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))


def test_profiles_present():
    names = {os.path.basename(p) for p in PROFILES}
    for need in ("bench_128x256x256_kernel_stats.txt", "cnn_fwd_bf16_128x256x256_traffic.txt",
                 "cnn_fwd_bf16_128x256x256_sq_counters.txt", "training_64x64_kernel_stats.txt"):
        assert need in names


@pytest.mark.parametrize("path", PROFILES, ids=os.path.basename)
def test_profile_names_its_commands(path):
    cmds = [v for k, v in PS.read_summary(path).items() if k.startswith("command")]
    assert cmds, "no command line"
    for c in cmds:
        assert c.startswith("rocprofv3 "), c
        prog = c.split(" -- ", 1)[1].split()
        assert prog[0] == "python3", c
        if prog[1] == "-m":
            mod = prog[2].replace(".", os.sep)
            assert os.path.exists(os.path.join(ROOT, mod + ".py")), c
        else:
            assert os.path.exists(os.path.join(ROOT, prog[1])), c
        assert "_work" not in c and "/root/" not in c, c


@pytest.mark.parametrize("path", [p for p in PROFILES if p.endswith(("_traffic.txt", "_sq_counters.txt"))],
                         ids=os.path.basename)
def test_counter_summary_matches_current_sources(path):
    base = os.path.basename(path)
    kind = next(k for k in PS.KERNEL_SOURCES if base.startswith(k + "_"))
    got = PS.read_summary(path).get("source_hash")
    assert got == PS.source_hash(kind), (
        "%s was taken from other sources of the %s kernel: take its counters again" % (base, kind))
