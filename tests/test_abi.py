"""C-ABI boundary checks that need no GPU: the library builds and loads,
exports every entry point declared in include/hac.h, rejects bad arguments,
and reports HAC_ENODEV when no gfx950 device is present."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1709_06816_amd as hac

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "hac.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(hac_\w+)\s*\(", src, re.M)))


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_library_exports_every_declared_symbol():
    lib = hac.load_library()
    names = _declared()
    assert set(names) == set(hac.EXPORTS), names
    for name in names:
        assert hasattr(lib, name), name


def test_null_arguments_rejected():
    lib = hac.load_library()
    assert lib.hac_destroy(None) == hac.HAC_OK
    assert lib.hac_sync(None) == hac.HAC_EINVAL
    assert lib.hac_set_option(None, 1, 1) == hac.HAC_EINVAL
    assert lib.hac_run(None, None, 4, 0, None, 0, None) == hac.HAC_EINVAL
    assert lib.hac_run_noalloc(None, None, 4, 0, None, 0, None) == hac.HAC_EINVAL
    assert lib.hac_batch(None, None, None, None, None, 0, None, None, 0, None) == hac.HAC_EINVAL
    assert lib.hac_create(0, None) == hac.HAC_EINVAL
    assert lib.hac_get_stats(None, None) == hac.HAC_EINVAL
    assert lib.hac_last_error(None) == b"no context"


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path")
def test_no_device_reports_enodev():
    lib = hac.load_library()
    h = ctypes.c_void_p()
    assert lib.hac_create(0, ctypes.byref(h)) == hac.HAC_ENODEV
    with pytest.raises(hac.HacError) as e:
        hac.Context(0)
    assert e.value.code == hac.HAC_ENODEV


def test_to_linkage_matrix_matches_scipy():
    """Host bookkeeping only: the records of the fp64 oracle converted to a
    SciPy linkage matrix equal SciPy's own on tie-free input."""
    from scipy.cluster.hierarchy import linkage as sp_linkage
    from scipy.spatial.distance import squareform
    import oracle
    rng = np.random.default_rng(3)
    x = rng.standard_normal((40, 3))
    d = np.sqrt(((x[:, None] - x[None]) ** 2).sum(-1))
    m = oracle.run_f64(d, "average")
    z = hac.to_linkage_matrix(m, 40)
    ref = sp_linkage(squareform(d, checks=False), "average")
    assert np.array_equal(z[:, :2], ref[:, :2])
    assert np.allclose(z[:, 2], ref[:, 2], rtol=1e-12)
    assert np.array_equal(z[:, 3], ref[:, 3])


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets the C
    compiler gives the structures of include/hac.h."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    structs = {"hac_stats": hac._Stats, "hac_server_stats": hac._ServerStats}
    lines = ["#include <stddef.h>", "#include <stdio.h>", "#include \"hac.h\"", "int main(void) {"]
    for cname, cls in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, stdout=subprocess.PIPE, text=True).stdout.split("\n")
    got = dict((" ".join(l.split()[:2]), int(l.split()[2])) for l in out if l.strip())
    for cname, cls in structs.items():
        assert got[cname + " size"] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got["%s %s" % (cname, f)] == getattr(cls, f).offset, (cname, f)


def test_linkage_names_match_header():
    """The binding's linkage names map onto the hac_linkage values of
    include/hac.h, one for each Table 1 row."""
    with open(os.path.join(ROOT, "include", "hac.h")) as f:
        src = f.read()
    body = re.search(r"typedef enum \{(.*?)\} hac_linkage;", src, re.S).group(1)
    declared = {m.group(1).lower(): int(m.group(2)) for m in re.finditer(r"HAC_(\w+)\s*=\s*(\d+)", body)}
    assert declared == hac.LINKAGES


def test_option_numbers_match_header():
    """Every hac_option of include/hac.h has the binding's OPT_* constant of
    the same name and value, and the binding defines no other."""
    with open(os.path.join(ROOT, "include", "hac.h")) as f:
        src = f.read()
    body = re.search(r"typedef enum \{(.*?)\} hac_option;", src, re.S).group(1)
    declared = {m.group(1): int(m.group(2)) for m in re.finditer(r"HAC_OPT_(\w+)\s*=\s*(\d+)", body)}
    bound = {k[len("OPT_"):]: v for k, v in vars(hac).items() if k.startswith("OPT_") and isinstance(v, int)}
    assert declared == bound
