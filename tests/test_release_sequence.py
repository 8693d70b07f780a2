"""Device code: every L2 write-back of a release is waited for before the
next memory instruction.

Publishing to another workgroup is "write this XCD's L2 back (buffer_wbl2),
wait for that write back, then store the flag".  The compiler emits that wait
only while the wave has other memory operations outstanding; after an
explicit wait for the wave's own stores it leaves it out, and the flag can
then reach a reader on another XCD before the data it publishes is in memory.
The kernels therefore wait explicitly after every release (release_agent /
release_system).  This test compiles every device source for gfx950 with the
library's flags and checks the generated assembly: after each buffer_wbl2, a
wait that includes vmcnt(0) comes before any branch or vector memory
instruction.  CPU only (hipcc cross-compiles)."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_1709_06816_amd import build as B

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_SOURCES = [s for s in B.SOURCES if s.endswith(".hip")]
MEM = re.compile(r"(global|flat|buffer|scratch)_(load|store|atomic)")


def _assemble(tmp):
    flags = [f for f in B.FLAGS if f not in ("-shared", "-fPIC", "-pthread")]
    procs, outs = [], []
    for src in HIP_SOURCES:
        out = os.path.join(tmp, os.path.basename(src) + ".s")
        cmd = [HIPCC, *flags, "--cuda-device-only", "-S", "-I", os.path.join(B.ROOT, "include"),
               "-I", os.path.join(B.HERE, "csrc"), "-o", out, src]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        outs.append(out)
    for p, src in zip(procs, HIP_SOURCES):
        log = p.communicate()[0]
        assert p.returncode == 0, "hipcc failed on %s:\n%s" % (src, log[-2000:])
    return outs


def unawaited_writebacks(lines):
    """Line numbers of buffer_wbl2 not followed by a vmcnt(0) wait before the
    next branch, memory instruction or end of function."""
    bad = []
    for i, line in enumerate(lines):
        t = line.strip()
        if not t.startswith("buffer_wbl2"):
            continue
        for u in lines[i + 1:]:
            u = u.strip()
            if u.startswith("s_waitcnt") and ("vmcnt(0)" in u or u == "s_waitcnt 0"):
                break
            if MEM.match(u) or u.startswith(("s_branch", "s_cbranch", "s_endpgm", "s_setpc", "s_barrier")):
                bad.append(i + 1)
                break
        else:
            bad.append(i + 1)
    return bad


def test_checker_flags_a_missing_wait():
    seq = ["buffer_wbl2 sc1", "s_waitcnt lgkmcnt(0)", "flat_store_dwordx2 v[8:9], v[6:7] sc1",
           "buffer_wbl2 sc1", "s_waitcnt vmcnt(0) expcnt(0) lgkmcnt(0)", "global_atomic_add v1, v2, s[8:9]",
           "buffer_wbl2 sc0 sc1", "s_cbranch_execz .LBB0_3", "s_waitcnt vmcnt(0)"]
    assert unawaited_writebacks(seq) == [1, 7]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_every_release_waits_for_its_write_back():
    tmp = tempfile.mkdtemp(prefix="hac_asm_")
    try:
        total, bad = 0, {}
        for path in _assemble(tmp):
            with open(path) as f:
                lines = f.read().split("\n")
            total += sum(1 for l in lines if l.strip().startswith("buffer_wbl2"))
            b = unawaited_writebacks(lines)
            if b:
                bad[os.path.basename(path)] = b[:10]
        assert total > 0, "no release found in the device code"
        assert not bad, "L2 write-backs not waited for: %s" % bad
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
