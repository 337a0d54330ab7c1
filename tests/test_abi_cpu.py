"""The C-ABI library loads, exports every symbol the public header declares,
and rejects malformed input before touching the GPU (runs without a GPU)."""
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2601_21990_amd.pdlpb as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdlpb.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdlpb_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    assert _declared() == sorted(P.EXPORTED)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in _declared():
        assert name in syms, name


def test_options_layout_matches_header():
    o = P.default_options()
    assert o.struct_size == P.C.sizeof(P.Options) == 160 and o.autotune == 1
    assert (o.eval_every, o.beta_sufficient, o.beta_necessary, o.beta_artificial, o.theta) == \
        (64, 0.2, 0.8, 0.36, 0.5)
    assert o.cross_sign == -1.0 and o.use_graphs == 1 and o.max_batch == 4096
    assert o.infeas_tol == -1.0 and o.dual_tol == -1.0
    assert P.C.sizeof(P.Delta) == 16


def test_options_offsets_match_the_c_compiler(tmp_path):
    """The ctypes mirror of pdlpb_options has the C compiler's field offsets."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    names = [f[0] for f in P.Options._fields_]
    src = tmp_path / "off.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "pdlpb.h"\nint main(void){\n'
                   + "".join(f'printf("%zu\\n", offsetof(pdlpb_options, {n}));\n' for n in names)
                   + 'printf("%zu\\n", sizeof(pdlpb_options));\nreturn 0;}\n')
    exe = tmp_path / "off"
    inc = os.path.join(os.path.dirname(__file__), "..", "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [getattr(P.Options, n).offset for n in names] + [P.C.sizeof(P.Options)]
    assert got == want


def _ctx(**over):
    kw = dict(m=2, n=3, row_ptr=[0, 2, 3], col_idx=[0, 2, 1], val=[1.0, 2.0, 3.0],
              c=np.zeros(3), b=np.zeros(2), sense=b"EL", l=np.zeros(3), u=np.ones(3))
    kw.update(over)
    return P.Context(**kw)


@pytest.mark.parametrize("over, msg", [
    (dict(col_idx=[0, 5, 1]), "column index out of range"),
    (dict(col_idx=[2, 0, 1]), "strictly increasing"),
    (dict(col_idx=[0, 0, 1]), "strictly increasing"),
    (dict(row_ptr=[1, 2, 3]), "row_ptr[0]"),
    (dict(m=3, row_ptr=[0, 3, 2, 3], col_idx=[0, 1, 2], b=np.zeros(3), sense=b"ELG"),
     "nondecreasing"),
    (dict(row_ptr=[0, 2, 1]), "exceeds nnz"),
    (dict(val=[1.0, np.nan, 3.0]), "finite"),
    (dict(c=np.array([0.0, np.inf, 0.0])), "objective"),
    (dict(b=np.array([np.nan, 0.0])), "right-hand side"),
    (dict(sense=b"EX"), "row sense"),
    (dict(l=np.array([0.0, 2.0, 0.0])), "lower bound above upper"),
    (dict(l=np.array([np.inf, 0.0, 0.0]), u=np.full(3, np.inf)), "wrong side"),
    (dict(u=np.array([1.0, np.nan, 1.0])), "NaN"),
])
def test_create_rejects_malformed_input(over, msg):
    with pytest.raises(P.PdlpbError) as e:
        _ctx(**over)
    assert e.value.code == P.EINVAL
    assert msg in str(e.value)


@pytest.mark.parametrize("over, msg", [
    (dict(row_ptr=[0, 2]), "row_ptr needs m + 1"),
    (dict(row_ptr=[0, 2, 3, 3]), "row_ptr needs m + 1"),
    (dict(col_idx=[0, 2]), "col_idx and val need"),
    (dict(val=[1.0, 2.0]), "col_idx and val need"),
    (dict(sense=b"E"), "sense needs m"),
    (dict(c=np.zeros(2)), "expected 3 entries"),
    (dict(b=np.zeros(3)), "expected 2 entries"),
])
def test_binding_checks_array_lengths_before_the_library_reads_them(over, msg):
    """The library takes plain pointers: an array shorter than the sizes say
    would be read past its end, so the binding refuses it first (no HIP call
    is made, which is why this runs without a GPU)."""
    with pytest.raises(ValueError) as e:
        _ctx(**over)
    assert msg in str(e.value)


@pytest.mark.parametrize("opt, msg", [
    (dict(precision=7), "precision"),
    (dict(eval_every=1), "eval_every"),
    (dict(cross_sign=0.5), "cross_sign"),
    (dict(tile_lanes=3), "tile_lanes"),
    (dict(tile_vec=3), "tile_vec"),
    (dict(step_size=-1.0), "step_size"),
    (dict(infeas_tol=float("nan")), "infeas_tol"),
    (dict(dual_tol=float("inf")), "dual_tol"),
    (dict(scaling=2), "scaling"),
    (dict(max_blocks=-1), "max_blocks"),
    (dict(dev_alloc=1), "dev_alloc and dev_free"),
    (dict(dev_free=1), "dev_alloc and dev_free"),
    (dict(eval_every=24, stop_every=1), "stop_every"),
    (dict(eval_every=24, stop_every=5), "stop_every"),
    (dict(eval_every=24, stop_every=48), "stop_every"),
    (dict(shared_start=2), "shared_start"),
    (dict(shared_start=-2), "shared_start"),
])
def test_create_rejects_bad_options(opt, msg):
    with pytest.raises(P.PdlpbError) as e:
        _ctx(options=P.default_options(**opt))
    assert e.value.code == P.EINVAL and msg in str(e.value)


def test_create_without_gpu_fails_cleanly():
    """On a machine without a GPU the first HIP call reports EDEVICE."""
    import ctypes
    try:
        n = P.C.c_int()
        have_gpu = ctypes.CDLL("libamdhip64.so").hipGetDeviceCount(ctypes.byref(n)) == 0 \
            and n.value > 0
    except OSError:
        have_gpu = False
    if have_gpu:
        pytest.skip("a GPU is present")
    with pytest.raises(P.PdlpbError) as e:
        _ctx()
    assert e.value.code == P.EDEVICE


def test_null_context_calls_are_rejected():
    assert P.lib.pdlpb_solve(None, 1e-4, 10) == P.EINVAL
    assert P.lib.pdlpb_set_batch(None, 1, None, None, None, None, 0, 0) == P.EINVAL
    assert P.lib.pdlpb_device_bytes(None) == 0
    assert P.lib.pdlpb_estimate_batch(None, None, 0, 10, None, None) == P.EINVAL
    assert P.lib.pdlpb_set_result_buffers(None, None, None, 0) == P.EINVAL
    P.lib.pdlpb_destroy(None)
