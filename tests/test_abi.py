"""The C ABI library loads and exports every entry point include/misa.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "misa.h")
LIB = os.path.join(ROOT, "paper_2107_07866_amd", "libmisa.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char \*)\s*\*?\s*(misa_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2107_07866_amd import build as B
        B.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("misa_create_lattice", "misa_set_potential_tables", "misa_compute_rho", "misa_compute_force",
                 "misa_step", "misa_set_state", "misa_get_state", "misa_destroy_lattice"):
        assert must in names
    assert len(names) >= 14


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2107_07866_amd import misa
    assert misa.declared_functions() == _declared()
    for n in _declared():
        assert callable(getattr(misa, n)), n


def test_descriptor_validation_without_gpu():
    """Invalid descriptors are rejected before any HIP call, with a message."""
    from paper_2107_07866_amd import misa as M
    cases = [
        dict(n_cells=(4, 16, 16), a=2.855, rc=5.0, delta=0.6, mass=55.845),    # 4 a < 2 (rc + 2 delta)
        dict(n_cells=(16, 16, 16), a=2.855, rc=5.0, delta=1.3, mass=55.845),   # delta >= a sqrt(3)/4
        dict(n_cells=(16, 16, 16), a=-1.0, rc=5.0, delta=0.6, mass=55.845),
        dict(n_cells=(16, 16, 16), a=2.855, rc=5.0, delta=0.6, mass=0.0),
        dict(n_cells=(16, 0, 16), a=2.855, rc=5.0, delta=0.6, mass=55.845),
    ]
    for c in cases:
        with pytest.raises(M.MisaError) as ei:
            M.misa_create_lattice(c["n_cells"], c["a"], c["rc"], c["delta"], c["mass"])
        assert ei.value.code == M.MISA_EINVAL
        assert M.misa_last_error(None)
    with pytest.raises(M.MisaError):
        M.misa_create_lattice((16, 16, 16), 2.855, 5.0, 0.6, 55.845, pair_precision=7)
    # only periodic boxes of one species (the descriptor's periodic[3] and ntypes)
    for kw in (dict(periodic=(1, 2, 1)), dict(periodic=(1, 1, -1)), dict(ntypes=2)):
        with pytest.raises(M.MisaError) as ei:
            M.misa_create_lattice((16, 16, 16), 2.855, 5.0, 0.6, 55.845, **kw)
        assert ei.value.code == M.MISA_EINVAL
        assert "periodic" in M.misa_last_error(None) or "ntypes" in M.misa_last_error(None)


def test_batch_limits_without_gpu():
    """A batch holds 1 .. 8192 boxes (its run-away work list is indexed through offsets
    staged in LDS); anything else is rejected before any HIP call."""
    from paper_2107_07866_amd import misa as M
    for n in (0, 8193):
        with pytest.raises(M.MisaError) as ei:
            M.misa_batch_create([(16, 16, 16)] * n, 2.855, 5.0, 0.6, 55.845)
        assert ei.value.code == M.MISA_EINVAL
        assert M.misa_batch_last_error(None)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2107_07866_amd import misa as M
    monkeypatch.setattr(M, "LIB_PATH", str(tmp_path / "libmisa.so"))
    with pytest.raises(ImportError):
        M._load()


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2107_07866_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f
