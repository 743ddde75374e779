"""The gfx950 code this library builds (CPU only: hipcc cross-compiles).

Compiles kernels.hip, server.hip and setup_dev.hip to device assembly with the
package's own flags and checks what the hot path relies on:

* every sweep kernel scatters with hardware float atomics
  (global/flat_atomic_add_f32 or _f64), never a compare-and-swap loop;
* no packed-FP32 instruction appears anywhere (the build disables them);
* the split worker's barriers (two waves, one barrier per batch) wait on the
  LDS counter only, never on the vector memory counter;
* the pipelined worker loop issues a lane's gathers for a ticket together:
  at least one unit's entries (4, or 8 for BF16) of agent-scope loads in a
  row with no wait between them, never one load per wait;
* the device-side setup forms the row weights with separate FP64 multiplies
  and adds (no fused multiply-add), so they equal the host's sums.
"""
import re
import shutil
import subprocess
from pathlib import Path

import pytest

from paper_1401_4780_amd import build as B

pytestmark = pytest.mark.skipif(not Path(B.HIPCC).exists() and not shutil.which("hipcc"),
                                reason="hipcc not available")


def _asm(src, tmp_path):
    out = tmp_path / (src + ".s")
    r = subprocess.run([B.HIPCC, *B.HIP_FLAGS, "-S", "--cuda-device-only", str(B.CSRC / src), "-o", str(out)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return out.read_text()


def _functions(asm):
    """{symbol: body} for every kernel in the assembly."""
    out = {}
    for mo in re.finditer(r"^(_Z\S+):\s*(?:;.*)?$", asm, re.M):
        name = mo.group(1)
        end = asm.find(".Lfunc_end", mo.end())
        out[name] = asm[mo.end():end]
    return out


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    tmp = tmp_path_factory.mktemp("isa")
    funcs = {}
    for src in ("kernels.hip", "server.hip", "setup_dev.hip"):
        funcs.update(_functions(_asm(src, tmp)))
    return funcs


def test_sweeps_use_hardware_float_atomics(kernels):
    sweeps = {k: v for k, v in kernels.items() if "sweep" in k and "kernel" in k}
    assert len(sweeps) >= 70, len(sweeps)
    for name, body in sweeps.items():
        assert re.search(r"(global|flat)_atomic_add_f(32|64)\b", body), name
        assert "cmpswap" not in body, name


def test_split_worker_barriers_wait_on_lds_only(kernels):
    """The split worker's two waves meet at a barrier per batch; the fences
    around it order LDS only, so no barrier waits on the vector memory
    counter (which would make the compute wave wait for its own atomics)."""
    split = {k: v for k, v in kernels.items() if "sweep_split_kernel" in k}
    assert len(split) >= 20, len(split)
    for name, body in split.items():
        lines = [ln.strip() for ln in body.splitlines()]
        bars = [i for i, ln in enumerate(lines) if ln.startswith("s_barrier")]
        assert len(bars) >= 4, (name, len(bars))  # two per role
        for i in bars:
            for ln in lines[max(0, i - 6):i]:
                assert not (ln.startswith("s_waitcnt") and "vmcnt" in ln), (name, ln)


def test_no_packed_fp32_instructions(kernels):
    for name, body in kernels.items():
        assert not re.search(r"\bv_pk_(add|mul|fma)_f32\b", body), name


def _lane_entries(name):
    """Entries one lane holds in the first chunk: U per unit x units per lane."""
    m = re.search(r"17sweep_pipe_kernelILi(\d)ELi(\d)ELi(\d+)E", name)
    if m:
        vk, g = int(m.group(1)), int(m.group(3))
        upl = 8 // g if g < 8 else 1
    else:  # the server's packed sweep: FP32 values, 16 / G units per lane
        m = re.search(r"srv_sweep_pipe_kernelILi(\d+)E", name)
        vk, g = 1, int(m.group(1))
        upl = 16 // g
    u = 8 if vk == 2 else 4  # BF16 units hold 8 entries, FP32/FP64 units 4
    return u * upl


def _unit_entries(name):
    m = re.search(r"17sweep_pipe_kernelILi(\d)E", name)
    return 8 if (m and int(m.group(1)) == 2) else 4


def test_pipelined_gathers_issue_back_to_back(kernels):
    """A lane's gathers for a ticket leave together, not one per wait."""
    pipe = {k: v for k, v in kernels.items() if "sweep_pipe_kernel" in k}
    assert len(pipe) >= 35
    for name, body in pipe.items():
        best = _longest_gather_run(body)
        # at least one unit's entries leave together: a lane whose units are
        # still arriving issues each unit's gathers as soon as that unit lands
        # (its waits retire unit data, not gathers); serialized gathers would
        # show runs of one
        want = min(_lane_entries(name), _unit_entries(name))
        assert best >= want, (name, best, want)


def _longest_gather_run(body):
    """Most coherent gathers (sc1 loads) issued with no wait between them
    that retires a gather.  Vector memory operations retire in issue order, so
    s_waitcnt vmcnt(N) retires all but the newest N outstanding ones; the
    queue is followed in program order through the listing."""
    queue, run, best = [], 0, 0
    for line in body.splitlines():
        t = line.strip()
        if re.match(r"(global|flat|buffer)_(load|store|atomic)", t):
            g = re.match(r"(global|flat)_load_dword(x2)?\b.*\bsc1\b", t) is not None
            queue.append(g)
            if g:
                run += 1
                best = max(best, run)
        else:
            w = re.match(r"s_waitcnt\b.*\bvmcnt\((\d+)\)", t)
            if w:
                keep = int(w.group(1))
                done, queue = (queue[:-keep], queue[-keep:]) if keep else (queue, [])
                if any(done):
                    run = 0
    return best


def test_device_setup_weights_are_unfused(kernels):
    scans = {k: v for k, v in kernels.items() if "scan_rows_kernel" in k}
    assert len(scans) == 3, sorted(kernels)
    for name, body in scans.items():
        assert "v_fma_f64" not in body and "v_fmac_f64" not in body, name
        assert "v_mul_f64" in body and "v_add_f64" in body, name
