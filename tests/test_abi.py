"""The C ABI on the host (no GPU needed): the library loads, exports every
function include/spmm.h declares, and rejects bad arguments before any HIP
call."""
import ctypes

import pytest

from paper_1803_08601_amd import native as nv


def test_header_symbols_exported():
    L = nv.lib()
    names = nv.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(nv._SIGS), "binding and header disagree"


def test_status_strings_and_version():
    assert nv.status_string(nv.SPMM_OK) == "ok"
    assert "invalid" in nv.status_string(nv.SPMM_ERR_INVALID)
    assert nv.status_string(12345) == "unknown status"
    assert nv.spmm_version().count(".") == 2


def _create(**kw):
    a = dict(out=ctypes.byref(ctypes.c_void_p()), rowptr=ctypes.c_void_p(8),
             colind=ctypes.c_void_p(8), m=10, k=10, nnz=20, n=4, ld=4, dtype=0, mode=0)
    a.update(kw)
    return nv.lib().spmm_plan_create(a["out"], a["rowptr"], a["colind"], a["m"], a["k"], a["nnz"],
                                     a["n"], a["ld"], a["dtype"], a["mode"], None)


@pytest.mark.parametrize("kw,status", [
    (dict(out=None), nv.SPMM_ERR_INVALID),
    (dict(m=-1), nv.SPMM_ERR_INVALID),
    (dict(n=-3), nv.SPMM_ERR_INVALID),
    (dict(nnz=-1), nv.SPMM_ERR_INVALID),
    (dict(ld=3), nv.SPMM_ERR_INVALID),
    (dict(n=0, ld=0), nv.SPMM_ERR_INVALID),
    (dict(dtype=7), nv.SPMM_ERR_UNSUPPORTED),
    (dict(mode=9), nv.SPMM_ERR_INVALID),
    (dict(rowptr=None), nv.SPMM_ERR_INVALID),
    (dict(colind=None), nv.SPMM_ERR_INVALID),
    (dict(m=2**31), nv.SPMM_ERR_UNSUPPORTED),
    # entry indices are int32 with chunk loops stepping past them: nnz is
    # capped 4096 below 2^31 - 1
    (dict(nnz=2**31 - 4096), nv.SPMM_ERR_UNSUPPORTED),
    (dict(nnz=2**31 - 1), nv.SPMM_ERR_UNSUPPORTED),
    (dict(k=0), nv.SPMM_ERR_INVALID),
])
def test_plan_create_rejects(kw, status):
    assert _create(**kw) == status
    assert nv.spmm_last_error()


def test_foreign_and_null_handles():
    L = nv.lib()
    bogus = ctypes.c_void_p(0x1234560)
    assert L.spmm_execute(bogus, None, None, None, None) == nv.SPMM_ERR_STATE
    assert L.spmm_plan_destroy(bogus) == nv.SPMM_ERR_STATE
    assert L.spmm_plan_destroy(None) == nv.SPMM_ERR_STATE
    assert L.spmm_plan_info_get(bogus, None) == nv.SPMM_ERR_STATE
    assert L.spmm_sddmm(bogus, None, None, None, None) == nv.SPMM_ERR_STATE
    assert L.spmm_execute_t(bogus, None, None, None, None) == nv.SPMM_ERR_STATE
    assert L.spmm_transpose_build(bogus, None) == nv.SPMM_ERR_STATE
    assert L.spmm_batch_run(bogus, None) == nv.SPMM_ERR_STATE
    assert L.spmm_batch_destroy(bogus) == nv.SPMM_ERR_STATE


def test_spmm_csr_noop_and_checks():
    L = nv.lib()
    # m == 0 or n == 0: no-op, no memory touched
    assert L.spmm_csr(None, None, None, None, None, 0, 5, 4, 4, None) == nv.SPMM_OK
    assert L.spmm_csr(None, None, None, None, None, 5, 5, 0, 1, None) == nv.SPMM_OK
    assert L.spmm_csr(None, None, None, None, None, 5, 5, 4, 2, None) == nv.SPMM_ERR_INVALID
    assert L.spmm_csr(None, None, None, None, None, -1, 5, 4, 4, None) == nv.SPMM_ERR_INVALID


def test_nnz_cap_on_every_plan_entry_point():
    L = nv.lib()
    cfg = nv.spmm_config(kernel=nv.SPMM_KERNEL_MERGE)
    out = ctypes.byref(ctypes.c_void_p())
    assert L.spmm_plan_create_config(out, ctypes.c_void_p(8), ctypes.c_void_p(8), 10, 10,
                                     2**31 - 4000, 4, 4, 0, ctypes.byref(cfg), None) \
        == nv.SPMM_ERR_UNSUPPORTED
    assert "2^31 - 4097" in nv.spmm_last_error()
    assert L.spmm_csr_validate(ctypes.c_void_p(8), ctypes.c_void_p(8), 10, 10, 2**31 - 2,
                               None) == nv.SPMM_ERR_UNSUPPORTED
    prob = nv.spmm_problem(8, 8, 8, 8, 8, 10, 10, 2**31 - 100, 4, 4)
    arr = (nv.spmm_problem * 1)(prob)
    assert L.spmm_batch_plan(out, arr, 1, 0, 0, None) == nv.SPMM_ERR_UNSUPPORTED


def test_csr_plan_info_checks():
    L = nv.lib()
    assert L.spmm_csr_plan_info(None, None, 5, 5, 4, 4, None, None) == nv.SPMM_ERR_INVALID


def test_config_struct_layout(tmp_path):
    """The ctypes structures match the C header's layout: a C program built
    against include/spmm.h prints every field's offset and each size."""
    import shutil
    import subprocess
    assert ctypes.sizeof(nv.spmm_config) == 36
    assert ctypes.sizeof(nv.spmm_problem) == 5 * 8 + 5 * 8
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"spmm_config": nv.spmm_config, "spmm_plan_info": nv.spmm_plan_info,
               "spmm_problem": nv.spmm_problem}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{nv.HEADER}"',
             "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    out = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(out[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset, f"{name}.{f}"


def _noalloc(**kw):
    a = dict(rowptr=ctypes.c_void_p(256), colind=ctypes.c_void_p(256),
             vals=ctypes.c_void_p(256), B=ctypes.c_void_p(256), C=ctypes.c_void_p(256),
             m=10, k=10, nnz=20, n=4, ld=4)
    a.update(kw)
    return nv.lib().spmm_csr_noalloc(a["rowptr"], a["colind"], a["vals"], a["B"], a["C"],
                                     a["m"], a["k"], a["nnz"], a["n"], a["ld"], None)


@pytest.mark.parametrize("kw,status", [
    (dict(m=-1), nv.SPMM_ERR_INVALID),
    (dict(ld=3), nv.SPMM_ERR_INVALID),
    (dict(nnz=-1), nv.SPMM_ERR_INVALID),
    (dict(nnz=2**31 - 1), nv.SPMM_ERR_UNSUPPORTED),
    (dict(C=None), nv.SPMM_ERR_INVALID),
    (dict(rowptr=None), nv.SPMM_ERR_INVALID),
    (dict(B=None), nv.SPMM_ERR_INVALID),
    # merge-based (nnz / m < 9.35): 4883 pieces of 1024 items with carry-out
    # rows of 4096 floats need 80 MB, more than the 64 MiB static scratch
    (dict(m=5_000_000, k=1, nnz=0, n=4096, ld=4096), nv.SPMM_ERR_UNSUPPORTED),
])
def test_noalloc_rejects_before_any_hip_call(kw, status):
    """spmm_csr_noalloc refuses bad sizes, null pointers and workspaces larger
    than its static scratch on the host (the pointers here are never used)."""
    assert _noalloc(**kw) == status
    assert nv.spmm_last_error()
    if kw.get("n") == 4096:
        assert "scratch" in nv.spmm_last_error()


def test_noalloc_degenerate_sizes_are_no_ops():
    assert _noalloc(m=0) == nv.SPMM_OK
    assert _noalloc(n=0, ld=1) == nv.SPMM_OK


def test_tune_cache_file_round_trip(tmp_path):
    """A loaded tune-cache entry is kept and written back unchanged; files that
    are missing, of another format or malformed are refused."""
    line = "0 100 100 900 8 8 20 0 0 0 0 1 1  1 4 8 2 2048 0 0 0 0  0.25"
    f = tmp_path / "t.txt"
    f.write_text("spmm-tune-cache 2\n" + line + "\n")
    nv.spmm_tune_cache_load(str(f))
    g = tmp_path / "u.txt"
    nv.spmm_tune_cache_save(str(g))
    rows = g.read_text().splitlines()
    assert rows[0] == "spmm-tune-cache 2"
    assert [r.split() for r in rows[1:]].count(line.split()) == 1
    bad = tmp_path / "bad.txt"
    for text in ("spmm-tune-cache 2\n1 2 3\n", "spmm-tune-cache 1\n" + line + "\n",
                 "something else\n",
                 "spmm-tune-cache 2\n" + line.replace(" 1 4 8 2", " 7 4 8 2") + "\n"):
        bad.write_text(text)
        with pytest.raises(nv.SpmmError) as ei:
            nv.spmm_tune_cache_load(str(bad))
        assert ei.value.status == nv.SPMM_ERR_INVALID
    with pytest.raises(nv.SpmmError):
        nv.spmm_tune_cache_load(str(tmp_path / "missing.txt"))


@pytest.mark.parametrize("kw", [dict(table=None), dict(out=None), dict(row_bytes=96), dict(row_bytes=1024),
                                dict(table_rows=0), dict(table_rows=3), dict(table_rows=2**32),
                                dict(steps=0), dict(steps=12), dict(threads=100),
                                dict(threads=0), dict(table=ctypes.c_void_p(8 + 4))])
def test_calibrate_gather_rejects(kw):
    """The gather calibration refuses bad arguments before any launch."""
    a = dict(table=ctypes.c_void_p(256), table_rows=1024, row_bytes=256, steps=64,
             out=ctypes.c_void_p(256), threads=2048)
    a.update(kw)
    assert nv.lib().spmm_calibrate_gather(a["table"], a["table_rows"], a["row_bytes"], a["steps"],
                                          a["out"], a["threads"], None) == nv.SPMM_ERR_INVALID
    assert nv.spmm_last_error()
