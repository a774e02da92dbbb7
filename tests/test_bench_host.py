"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
bytes behind the roofline figures, the send shares they assume (checked
against the library's source), and the rule that measured traffic is
reported only for the sources it was measured on."""
import json
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_send_shares_match_the_library():
    src = open(os.path.join(ROOT, "paper_2509_01742_amd", "csrc", "k_access.hip")).read()
    m = re.search(r"constexpr uint32_t (kShareFinish = \d+(?:, kShare\w+ = \d+)*);", src)
    assert m, "share constants not found"
    lib = {k: int(v) for k, v in re.findall(r"kShare(\w+) = (\d+)", m.group(1))}
    names = {"Finish": "finish", "Group": "group", "Resolve": "resolve", "Place": "place", "Compose": "compose"}
    assert {names[k]: v for k, v in lib.items()} == bench.SEND_SLICES_64
    assert bench.FETCH_SEND_FRACTION == (64 - sum(lib.values())) / 64


SZ_HOST = {"page_bytes": 1024, "B": 2105344, "Z": 14, "K": 421068, "M": 1684276, "vs": 64, "host": 1}


def test_algorithmic_bytes():
    sz_dev = dict(SZ_HOST, host=0)
    n, npad, q = 1 << 24, 1 << 24, 4096
    roles = 2 * q * SZ_HOST["M"] / SZ_HOST["B"]
    assert bench.kernel_bytes("sort_global", SZ_HOST, n, npad, q, roles) == (16 * npad, "hbm")
    assert bench.kernel_bytes("expand", SZ_HOST, n, npad, q, roles) == (16 * SZ_HOST["B"] * SZ_HOST["Z"], "hbm")
    assert bench.kernel_bytes("page_writeout", SZ_HOST, n, npad, q, roles) == (SZ_HOST["M"] * 1024, "host_link")
    # the fetch reads about 2 (1 - alpha) pages per command, and writes its share of the previous batch's pages
    assert bench.kernel_bytes("acc_fetch", SZ_HOST, n, npad, q, roles) == (roles * 1024, "host_link")
    share = bench.FETCH_SEND_FRACTION * 63 / 64
    per, bound = bench.kernel_bytes("acc_fetch", SZ_HOST, n, npad, q, roles, share)
    assert bound == "host_link_duplex" and per == pytest.approx(roles * 1024 * (1 + share))
    assert bench.kernel_bytes("acc_fetch", sz_dev, n, npad, q, roles) == (2 * q * 1024, "hbm")
    assert bench.kernel_bytes("acc_resolve", SZ_HOST, n, npad, q, roles) == (None, None)


def test_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    """A tree whose sources hash to the values recorded with the counters
    reports the kernel's measured bytes; one byte changed in a source, and
    it reports none."""
    import hashlib

    for d in ("profiles", os.path.join("paper_2509_01742_amd", "csrc")):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d)
    prof_path = tmp_path / "profiles" / "traffic_plain_omap_n24_v64.json"
    prof = json.load(open(prof_path))
    csrc = tmp_path / "paper_2509_01742_amd" / "csrc"
    prof["sources"] = {fn: hashlib.sha256(open(csrc / fn, "rb").read()).hexdigest()[:16] for fn in prof["sources"]}
    json.dump(prof, open(prof_path, "w"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    got = bench.measured_traffic("acc_fetch", "host")
    assert got is not None and got["bytes"] == got["fetch_bytes"] + got["write_bytes"] > 0
    with open(csrc / "k_access.hip", "a") as f:
        f.write("\n")
    assert bench.measured_traffic("acc_fetch", "host") is None
