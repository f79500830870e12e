"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/nnqmd.h, reports the same weight layout as the oracle, and
rejects bad model descriptions on the host."""
import ctypes as C
import os
import re

import pytest

import oracle
from paper_2303_08169_amd import binding as B
from synth import CONFIGS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "nnqmd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nq_[a-z_]+)\s*\(", text)))


def test_header_lists_the_bound_entry_points():
    assert _declared() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = B.lib()
    for name in _declared():
        assert hasattr(L, name), name


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_weight_layout_matches_oracle(name, prec):
    model = CONFIGS[name].model
    segs, total = B.weight_layout(B.make_desc(model, prec))
    ref = [(a, b) for _, a, b in oracle.weight_segments(model)]
    assert segs == ref
    assert total == sum(a * b for a, b in ref)


def test_bad_descriptions_are_rejected_on_the_host():
    L = B.lib()
    base = CONFIGS["nh3_1024_l2"].model
    for field, value in [("lmax", 3), ("channels", 12), ("n_layers", 0), ("n_species", 9)]:
        d = B.make_desc(base)
        setattr(d, field, value)
        nseg, ntot = C.c_int32(0), C.c_int64(0)
        st = L.nq_model_weight_layout(C.byref(d), None, 0, C.byref(nseg), C.byref(ntot))
        assert st != 0, field
        assert L.nq_last_error(None).decode()
    d = B.make_desc(base)
    d.latent[0] = 128  # last latent width must equal the two-body output width
    nseg, ntot = C.c_int32(0), C.c_int64(0)
    assert L.nq_model_weight_layout(C.byref(d), None, 0, C.byref(nseg), C.byref(ntot)) == -1


def test_status_strings():
    L = B.lib()
    for s in B.STATUS:
        assert L.nq_status_str(s)
