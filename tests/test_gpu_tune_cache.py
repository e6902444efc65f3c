"""The tile-shape cache file ($DD_TUNE_CACHE) is keyed by GPU architecture.

A line written for another architecture must not be applied on this GPU;
the same line under this GPU's architecture must be.  Each case runs in a
fresh process because the library reads the file once, at first use.
"""
import os
import subprocess
import sys
import textwrap

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent("""
    import json, math, sys
    sys.path.insert(0, {root!r})
    import torch
    import paper_1107_2516_amd as dd
    import synth
    b = synth.Band(256, 1510.0, 296.0 / 256, 64e-6)
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, synth.dm_grid(100, 0.5))
    nsamp = plan.max_shift + 5000
    print(json.dumps(plan.tile_for(torch.float32, nsamp)))
""")


def _tile_with_cache(tmp_path, arch):
    import paper_1107_2516_amd as dd
    import synth
    b = synth.Band(256, 1510.0, 296.0 / 256, 64e-6)
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, synth.dm_grid(100, 0.5))
    nsamp = plan.max_shift + 5000
    log2 = (nsamp - 1).bit_length()
    path = tmp_path / f"tune_{arch}.txt"
    # variant 0, 8 DMs per wave, 4 waves, 8 samples per lane, 8 channels per stage
    path.write_text(f"{arch} {dd.DD_F32} 256 100 {plan.max_shift} {log2} 0 8 4 8 8\n")
    env = dict(os.environ, DD_TUNE_CACHE=str(path))
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT)], env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    import json
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_cache_line_of_this_architecture_applies(tmp_path):
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    assert _tile_with_cache(tmp_path, arch)["variant"] == 0


def test_cache_line_of_another_architecture_is_ignored(tmp_path):
    assert _tile_with_cache(tmp_path, "gfx000")["variant"] != 0
