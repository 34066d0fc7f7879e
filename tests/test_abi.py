"""The C ABI library loads and exports every symbol that include/scqr.h declares; argument
errors are returned synchronously (CPU only: no call here reaches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scqr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(scqr_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    import paper_1809_11085_amd as scqr
    if not os.path.exists(scqr.LIB_PATH):
        from paper_1809_11085_amd import build
        build.build()
    return scqr.lib()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ["scqr_qr", "scqr_gram", "scqr_trsm", "scqr_qr_batched", "scqr_qr_backward",
                 "scqr_workspace_bytes", "scqr_status_string", "scqr_default_opts"]:
        assert must in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings_and_defaults(L):
    import paper_1809_11085_amd as scqr
    for s in range(8):
        assert scqr.status_string(s).startswith("SCQR")
    o = scqr._Opts()
    L.scqr_default_opts(ctypes.byref(o))
    assert o.schedule == 1 and o.shift_mode == 0 and o.max_passes == 6 and o.trace is None
    assert "gfx950" in scqr.build_info()


def test_workspace_bytes_and_invalid_shapes(L):
    import paper_1809_11085_amd as scqr
    sz = ctypes.c_size_t()
    assert L.scqr_workspace_bytes(1 << 22, 64, None, None, ctypes.byref(sz)) == scqr.OK
    assert sz.value > 64 * 64 * 8
    assert L.scqr_workspace_bytes(10, 20, None, None, ctypes.byref(sz)) == scqr.E_INVALID
    assert L.scqr_workspace_bytes(1000, 0, None, None, ctypes.byref(sz)) == scqr.E_INVALID
    assert L.scqr_workspace_bytes(1000, 257, None, None, ctypes.byref(sz)) == scqr.E_INVALID


def test_synchronous_argument_errors(L):
    import paper_1809_11085_amd as scqr
    P = 0x100000  # never dereferenced: every call below fails validation first
    info = ctypes.c_void_p(P)
    # m < n
    assert L.scqr_qr(None, 5, 10, P, 10, None, P, 10, P, 10, P, 1 << 30, None, info) == scqr.E_INVALID
    # n above the maximum
    assert L.scqr_qr(None, 5000, 300, P, 300, None, P, 300, P, 300, P, 1 << 30, None, info) == scqr.E_UNSUPPORTED
    # leading dimension too small
    assert L.scqr_qr(None, 5000, 30, P, 20, None, P, 30, P, 30, P, 1 << 30, None, info) == scqr.E_INVALID
    # null pointers
    assert L.scqr_qr(None, 5000, 30, None, 30, None, P, 30, P, 30, P, 1 << 30, None, info) == scqr.E_INVALID
    # bad option
    o = scqr._Opts()
    L.scqr_default_opts(ctypes.byref(o))
    o.max_passes = 0
    assert L.scqr_qr(None, 5000, 30, P, 30, None, 0x900000000, 30, 0x800000000, 30, 0x700000000,
                     1 << 30, ctypes.byref(o), info) == scqr.E_INVALID
    # workspace too small
    assert L.scqr_qr(None, 5000, 30, P, 30, None, 0x900000000, 30, 0x800000000, 30, 0x700000000,
                     16, None, info) == scqr.E_WORKSPACE
    # R overlapping X
    assert L.scqr_qr(None, 5000, 30, P, 30, None, 0x900000000, 30, P + 8, 30, 0x700000000,
                     1 << 30, None, info) == scqr.E_INVALID
    # FP32-first with an oblique B is not supported
    o2 = scqr._Opts()
    L.scqr_default_opts(ctypes.byref(o2))
    o2.precision = 1
    spd = scqr._SpdOp()
    spd.kind = 1
    spd.diag = 0x600000000
    spd.off = 0x610000000
    assert L.scqr_qr(None, 5000, 30, P, 30, ctypes.byref(spd), 0x900000000, 30, 0x800000000, 30,
                     0x700000000, 1 << 30, ctypes.byref(o2), info) == scqr.E_UNSUPPORTED
    # the summation-depth shift is Euclidean only
    o3 = scqr._Opts()
    L.scqr_default_opts(ctypes.byref(o3))
    o3.shift_mode = 4
    assert L.scqr_qr(None, 5000, 30, P, 30, ctypes.byref(spd), 0x900000000, 30, 0x800000000, 30,
                     0x700000000, 1 << 30, ctypes.byref(o3), info) == scqr.E_UNSUPPORTED
    o3.shift_mode = 5
    assert L.scqr_qr(None, 5000, 30, P, 30, None, 0x900000000, 30, 0x800000000, 30,
                     0x700000000, 1 << 30, ctypes.byref(o3), info) == scqr.E_INVALID
    # minimum-traffic passes: n <= 32 and B = I only; the flag is 0 or 1; not batched
    o4 = scqr._Opts()
    L.scqr_default_opts(ctypes.byref(o4))
    assert o4.recompute == 0
    o4.recompute = 1
    assert L.scqr_qr(None, 5000, 33, P, 33, None, 0x900000000, 33, 0x800000000, 33,
                     0x700000000, 1 << 30, ctypes.byref(o4), info) == scqr.E_UNSUPPORTED
    assert L.scqr_qr(None, 5000, 30, P, 30, ctypes.byref(spd), 0x900000000, 30, 0x800000000, 30,
                     0x700000000, 1 << 30, ctypes.byref(o4), info) == scqr.E_UNSUPPORTED
    sz4 = ctypes.c_size_t()
    arr = lambda v: (ctypes.c_int64 * len(v))(*v)  # noqa: E731
    assert L.scqr_batched_workspace_bytes(1, arr([1000]), arr([8]), ctypes.byref(o4), None,
                                          ctypes.byref(sz4)) == scqr.E_UNSUPPORTED
    o4.recompute = 2
    assert L.scqr_qr(None, 5000, 30, P, 30, None, 0x900000000, 30, 0x800000000, 30,
                     0x700000000, 1 << 30, ctypes.byref(o4), info) == scqr.E_INVALID
    # CSR B: row pointers required; values and columns when nnz > 0; nnz >= 0
    csr = scqr._SpdOp()
    csr.kind = 2
    csr.nnz = 10
    args = (None, 5000, 30, P, 30, ctypes.byref(csr), 0x900000000, 30, 0x800000000, 30, 0x700000000, 1 << 30)
    assert L.scqr_qr(*args, None, info) == scqr.E_INVALID  # no row_ptr
    csr.row_ptr, csr.col = 0x600000000, 0x610000000
    assert L.scqr_qr(*args, None, info) == scqr.E_INVALID  # no val
    csr.val, csr.nnz = 0x620000000, -1
    assert L.scqr_qr(*args, None, info) == scqr.E_INVALID  # negative nnz
    csr.nnz = 10
    o5 = scqr._Opts()
    L.scqr_default_opts(ctypes.byref(o5))
    o5.precision = 1
    assert L.scqr_qr(*args, ctypes.byref(o5), info) == scqr.E_UNSUPPORTED
    csr.kind = 3
    assert L.scqr_qr(*args, None, info) == scqr.E_INVALID  # unknown kind
    csr.kind = 2
    sz5 = ctypes.c_size_t()
    assert L.scqr_workspace_bytes(5000, 30, ctypes.byref(csr), None, ctypes.byref(sz5)) == scqr.OK
    sz6 = ctypes.c_size_t()
    assert L.scqr_workspace_bytes(5000, 30, None, None, ctypes.byref(sz6)) == scqr.OK
    assert sz5.value > sz6.value  # the oblique first pass keeps a second (Euclidean) Gram
    # backward: dX aliasing Q
    assert L.scqr_qr_backward(None, 5000, 30, P, 30, 0x800000000, 30, None, 30, None, 30, P, 30,
                              0x700000000, 1 << 30) == scqr.E_INVALID
    # batched: negative batch
    assert L.scqr_qr_batched(None, -1, None, None, None, None, None, None, None, None, None, 0, None, None,
                             None) == scqr.E_INVALID
    assert L.scqr_qr_batched(None, 0, None, None, None, None, None, None, None, None, None, 0, None, None,
                             None) == scqr.OK


def _arr(t, v):
    return (t * len(v))(*v)


def test_batched_leading_dimensions_and_tuning_validation(L):
    # per-instance leading dimensions: ld_i >= n_i, Q_i == X_i only with ldq_i == ldx_i; tuning
    # values checked; every failure is synchronous (no device pointer is dereferenced)
    import paper_1809_11085_amd as scqr
    I64, VP = ctypes.c_int64, ctypes.c_void_p
    ms, ns = _arr(I64, [5000, 3000]), _arr(I64, [30, 64])
    X = _arr(VP, [0x100000000, 0x200000000])
    Q = _arr(VP, [0x300000000, 0x400000000])
    R = _arr(VP, [0x500000000, 0x500100000])
    info, ws = 0x600000000, 0x700000000
    sz = ctypes.c_size_t()
    assert L.scqr_batched_workspace_bytes(2, ms, ns, None, None, ctypes.byref(sz)) == scqr.OK
    big = 1 << 34

    def call(ldx=None, ldq=None, ldr=None, Qp=Q, tune=None, wsb=big):
        return L.scqr_qr_batched(None, 2, ms, ns, X, ldx, Qp, ldq, R, ldr, ws, wsb, None, tune, info)

    assert call(ldx=_arr(I64, [29, 64])) == scqr.E_INVALID
    assert call(ldq=_arr(I64, [30, 63])) == scqr.E_INVALID
    assert call(ldr=_arr(I64, [30, 10])) == scqr.E_INVALID
    assert call(wsb=16) == scqr.E_WORKSPACE
    # in place with different leading dimensions of X_0 and Q_0
    assert call(ldx=_arr(I64, [32, 64]), ldq=_arr(I64, [30, 64]), Qp=X) == scqr.E_INVALID
    # a strided X_1 that would run into Q_1
    assert L.scqr_qr_batched(None, 2, ms, ns, X, _arr(I64, [30, 1 << 22]), _arr(VP, [0x300000000, 0x200100000]),
                             None, R, None, ws, big, None, None, info) == scqr.E_INVALID
    t = scqr._Tuning()
    t.panel_rows[3] = 64   # 64-row panels exist for widths <= 64 only
    assert call(tune=ctypes.byref(t)) == scqr.E_INVALID
    t = scqr._Tuning()
    t.panel_rows[0] = 48
    assert call(tune=ctypes.byref(t)) == scqr.E_INVALID
    t = scqr._Tuning()
    t.rows_per_task[2] = -5
    assert L.scqr_batched_workspace_bytes(2, ms, ns, None, ctypes.byref(t), ctypes.byref(sz)) == scqr.E_INVALID
    # a larger leading dimension is accepted by the planner (the workspace does not depend on it)
    t = scqr._Tuning()
    t.rows_per_task[1] = 100   # rounded up to 128
    t.panel_rows[2] = 64
    assert L.scqr_batched_workspace_bytes(2, ms, ns, None, ctypes.byref(t), ctypes.byref(sz)) == scqr.OK


def test_batched_plan_host_side(L):
    # plan creation validates like scqr_qr_batched and reports the tuning in effect; no device
    # work happens before upload
    import paper_1809_11085_amd as scqr
    I64, VP = ctypes.c_int64, ctypes.c_void_p
    ms, ns = _arr(I64, [200000, 3000, 70000]), _arr(I64, [64, 128, 16])
    X = _arr(VP, [0x100000000, 0x200000000, 0x280000000])
    Q = _arr(VP, [0x300000000, 0x400000000, 0x480000000])
    R = _arr(VP, [0x500000000, 0x500100000, 0x500200000])
    sz = ctypes.c_size_t()
    t = scqr._Tuning()
    t.rows_per_task[2] = 5000   # rounded up to a multiple of 64
    t.panel_rows[2] = 64
    assert L.scqr_batched_workspace_bytes(3, ms, ns, None, ctypes.byref(t), ctypes.byref(sz)) == scqr.OK
    h = ctypes.c_void_p()
    assert L.scqr_batched_plan_create(3, ms, ns, X, None, Q, None, R, None, 0x700000000, 16, None,
                                      ctypes.byref(t), 0x600000000, ctypes.byref(h)) == scqr.E_WORKSPACE
    assert not h.value
    assert L.scqr_batched_plan_create(3, ms, ns, X, None, Q, None, R, None, 0x700000000, sz.value, None,
                                      ctypes.byref(t), 0x600000000, ctypes.byref(h)) == scqr.OK
    got = scqr._Tuning()
    nt = (ctypes.c_int32 * 5)()
    assert L.scqr_batched_plan_tuning(h, ctypes.byref(got), nt) == scqr.OK
    assert got.rows_per_task[2] == 5056 and got.panel_rows[2] == 64 and got.panel_rows[0] == 32
    # 200000 rows in tasks of at most 5056 rows, split evenly: 40 tasks of 5056 rows (to 64);
    # 70000 rows at the default 1024: 69 tasks; 3000 rows: 3 tasks
    assert list(nt) == [69, 0, 40, 3, 0]
    assert got.rows_per_task[0] == 1024 and got.rows_per_task[3] == 1024   # default: >= 1024 rows
    # run before upload is refused
    assert L.scqr_batched_plan_run(h, None) == scqr.E_INVALID
    assert L.scqr_batched_plan_destroy(h) == scqr.OK
    assert L.scqr_batched_plan_destroy(None) == scqr.OK
    assert L.scqr_batched_plan_run(None, None) == scqr.E_INVALID


def test_product_path_has_no_fallback(monkeypatch, tmp_path):
    import paper_1809_11085_amd as scqr
    monkeypatch.setattr(scqr, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(scqr, "_lib", None)
    with pytest.raises(RuntimeError):
        scqr.lib()


def test_profile_read_arguments(L):
    # validation and an empty record need no device
    import paper_1809_11085_amd as scqr
    cnt = ctypes.c_int32(-1)
    assert L.scqr_profile_read(None, 0, None) == scqr.E_INVALID
    assert L.scqr_profile_read(None, -1, ctypes.byref(cnt)) == scqr.E_INVALID
    assert L.scqr_profile_read(None, 4, ctypes.byref(cnt)) == scqr.E_INVALID
    assert L.scqr_profile_enable(0) == scqr.OK
    assert L.scqr_profile_read(None, 0, ctypes.byref(cnt)) == scqr.OK and cnt.value == 0


def test_workspace_sizes_of_batched_and_adjoint(L):
    # host-side planning only: validation and sizes, no device memory touched
    import paper_1809_11085_amd as scqr
    sz = ctypes.c_size_t()

    def arr(v):
        return (ctypes.c_int64 * len(v))(*v)

    ms, ns = [20000, 5000, 3001, 100000], [64, 16, 128, 256]
    assert L.scqr_batched_workspace_bytes(4, arr(ms), arr(ns), None, None, ctypes.byref(sz)) == scqr.OK
    full = sz.value
    assert full % 256 == 0 and full > 0
    assert L.scqr_batched_workspace_bytes(3, arr(ms[:3]), arr(ns[:3]), None, None, ctypes.byref(sz)) == scqr.OK
    assert 0 < sz.value < full
    # FIXED3 keeps three factor slots per instance instead of max_passes
    o = scqr._Opts()
    L.scqr_default_opts(ctypes.byref(o))
    o.schedule = scqr.SCHEDULES["fixed3"]
    assert L.scqr_batched_workspace_bytes(4, arr(ms), arr(ns), ctypes.byref(o), None, ctypes.byref(sz)) == scqr.OK
    assert sz.value < full
    assert L.scqr_batched_workspace_bytes(0, None, None, None, None, ctypes.byref(sz)) == scqr.OK
    assert L.scqr_batched_workspace_bytes(-1, None, None, None, None, ctypes.byref(sz)) == scqr.E_INVALID
    assert L.scqr_batched_workspace_bytes(2, None, arr([4, 4]), None, None, ctypes.byref(sz)) == scqr.E_INVALID
    assert L.scqr_batched_workspace_bytes(1, arr([10]), arr([20]), None, None, ctypes.byref(sz)) == scqr.E_INVALID
    assert L.scqr_batched_workspace_bytes(1, arr([1000]), arr([0]), None, None, ctypes.byref(sz)) == scqr.E_INVALID
    assert L.scqr_batched_workspace_bytes(1, arr([1000]), arr([257]), None, None, ctypes.byref(sz)) == \
        scqr.E_UNSUPPORTED
    assert L.scqr_batched_workspace_bytes(1, arr([1000]), arr([8]), None, None, None) == scqr.E_INVALID
    o.max_passes = 0
    o.schedule = scqr.SCHEDULES["adaptive"]
    assert L.scqr_batched_workspace_bytes(1, arr([1000]), arr([8]), ctypes.byref(o), None, ctypes.byref(sz)) == \
        scqr.E_INVALID

    assert L.scqr_backward_workspace_bytes(100000, 64, ctypes.byref(sz)) == scqr.OK and sz.value > 0
    small = sz.value
    assert L.scqr_backward_workspace_bytes(100000, 256, ctypes.byref(sz)) == scqr.OK and sz.value > small
    assert L.scqr_backward_workspace_bytes(10, 20, ctypes.byref(sz)) == scqr.E_INVALID
    assert L.scqr_backward_workspace_bytes(1000, 0, ctypes.byref(sz)) == scqr.E_INVALID
    assert L.scqr_backward_workspace_bytes(1000, 257, ctypes.byref(sz)) == scqr.E_INVALID
    assert L.scqr_backward_workspace_bytes(1000, 8, None) == scqr.E_INVALID


def test_noalloc_validation_without_device(L):
    # argument errors and shapes whose workspace exceeds the static scratch are rejected before
    # any HIP call
    import paper_1809_11085_amd as scqr
    P = 0x100000
    info = ctypes.c_void_p(P)
    assert L.scqr_qr_noalloc(None, 5, 10, P, 10, None, P, 10, P, 10, None, info) == scqr.E_INVALID
    assert L.scqr_qr_noalloc(None, 5000, 300, P, 300, None, P, 300, P, 300, None, info) == scqr.E_UNSUPPORTED
    assert L.scqr_qr_noalloc(None, 5000, 30, P, 20, None, P, 30, P, 30, None, info) == scqr.E_INVALID
    assert L.scqr_qr_noalloc(None, 5000, 30, P, 30, None, P, 30, P, 30, None, None) == scqr.E_INVALID
    o = scqr._Opts()
    L.scqr_default_opts(ctypes.byref(o))
    o.schedule = 9
    assert L.scqr_qr_noalloc(None, 5000, 30, P, 30, None, P, 30, P, 30, ctypes.byref(o), info) == scqr.E_INVALID
    # n = 128 and 256 need more than the scratch holds
    for n in (128, 256):
        assert L.scqr_qr_noalloc(None, 1 << 20, n, P, n, None, 0x900000000, n, 0x800000000, n, None,
                                 info) == scqr.E_WORKSPACE
    # every shape up to n = 64 fits, Euclidean or oblique
    sz = ctypes.c_size_t()
    spd = scqr._SpdOp()
    spd.kind = 1
    for n in (1, 16, 33, 64):
        for Bp in (None, ctypes.byref(spd)):
            assert L.scqr_workspace_bytes(1 << 30, n, Bp, None, ctypes.byref(sz)) == scqr.OK
            assert sz.value <= scqr.NOALLOC_SCRATCH_BYTES


def test_autotune_candidates_and_cache_io(tmp_path, monkeypatch):
    # host logic of the batched autotuner: candidate sets and the JSON cache round trip
    from paper_1809_11085_amd import autotune
    c64 = autotune.candidates(2, [(20000, 64), (50000, 60)])
    assert (0, 32) in c64 and (0, 64) in c64 and all(r < 100000 for r, _ in c64)
    c128 = autotune.candidates(3, [(3000, 128)])
    assert all(p == 0 for _, p in c128) and all(r < 6000 for r, _ in c128)
    monkeypatch.setenv("SCQR_AUTOTUNE_CACHE", str(tmp_path / "x" / "c.json"))
    p = autotune.cache_path()
    assert p == str(tmp_path / "x" / "c.json")
    assert autotune._load_cache(p) == {}
    autotune._store_cache(p, {"k": {"rows_per_task": 2048, "panel_rows": 32}})
    assert autotune._load_cache(p)["k"]["rows_per_task"] == 2048


def test_struct_layouts_match_header(tmp_path):
    # the ctypes mirrors of scqr_opts, scqr_info, scqr_spd_op and scqr_batched_tuning have the
    # C layout of include/scqr.h (sizes and the offset of every field), checked with the host C
    # compiler
    import shutil
    import subprocess

    import paper_1809_11085_amd as scqr
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    mirrors = {"scqr_opts": scqr._Opts, "scqr_info": scqr._Info, "scqr_spd_op": scqr._SpdOp,
               "scqr_batched_tuning": scqr._Tuning, "scqr_kernel_stat": scqr._KernelStat}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "scqr.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname}.{f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for cname, py in mirrors.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert int(out[f"{cname}.{f[0]}"]) == getattr(py, f[0]).offset, (cname, f[0])
