"""Host-side tests of the C ABI: the library loads, exports every declared
entry point, validates arguments and builds self-checked line-solve tables.
No HIP call is made (etd_rdp_init is host-only)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2001_11220_amd import etd
    return etd


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(etd_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    etd = _lib()
    names = _declared_functions()
    assert "etd_rdp_init" in names and "etd_rdp_step" in names
    for n in sorted(names):
        assert hasattr(etd.lib, n), n


def _init(shape, bcs, D=(0.1, 0.2), k=0.01, model="brusselator", params=None, h=None, scheme="rdp",
          lines_per_wave="auto", precision="f64"):
    etd = _lib()
    params = params if params is not None else {"a": 1.0, "b": 3.0}
    return etd.EtdRdp(shape, bcs, D, k, model, params, h=h, scheme=scheme, lines_per_wave=lines_per_wave,
                      precision=precision)


@pytest.mark.parametrize("bc", ["dirichlet", "neumann", "periodic"])
def test_tables_build_for_every_line_length(bc):
    """Every line length 1..1024 builds its tables (each passes the table
    builder's residual self-check of the chunked algorithm).  Regular
    lengths split into C <= 64 equal chunks of m <= 8 rows; the others
    ("general" lines) into m = ceil(n/64) rows per chunk and C = ceil(n/m)
    chunks, the last one shorter when m does not divide n."""
    nmin = {"dirichlet": 1, "neumann": 2, "periodic": 3}[bc]
    for n in range(nmin, 1025):
        p = _init((n,), (bc,), D=(0.5, 3.0), k=0.3)
        m, C = p.line_split(1)
        regular = any(n % q == 0 and n // q <= 64 for q in range(1, 9))
        if regular:
            assert m * C == n and C <= 64 and 1 <= m <= 8, (n, m, C)
            assert not p.pass_kernel(1).startswith("kr_")
        else:
            assert m == -(-n // 64) and C == -(-n // m) and (C - 1) * m < n <= C * m, (n, m, C)
            assert p.pass_kernel(1).startswith("kr_last<"), p.pass_kernel(1)
        p.close()


def test_lines_per_wave_option():
    from paper_2001_11220_amd import etd
    bcs = ("periodic", "neumann", "dirichlet")
    # automatic, on passes with at least 8192 lines: eight lines per
    # wavefront for n = 8 m, else four for n = 16 m, else two for n = 32 m
    # (m = 2..8 each)
    big = _init((256, 256, 160), bcs)
    assert [big.line_split(a) for a in (1, 2, 3)] == [(8, 32), (8, 32), (5, 32)]
    assert big.pass_kernel(1) == "k_first_pair<8, 16, 2, true, false, double>"
    small = _init((256, 24, 10), bcs)  # 240 lines: one line per wavefront
    assert small.line_split(1) == (4, 64) and small.pass_kernel(1) == "k_first<4, 2, 16, false, double>"
    tiny = _init((256, 12, 10), bcs)  # 120 lines (latency-bound): two
    assert tiny.line_split(1) == (8, 32)
    tiny.close()
    two = _init((256, 12, 10), bcs, lines_per_wave=2)
    assert two.line_split(1) == (8, 32) and two.pass_kernel(1) == "k_first_pair<8, 16, 2, false, false, double>"
    assert two.line_split(2) == (1, 12)  # lengths that are not 32 m keep one line
    one = _init((256, 192, 160), bcs, lines_per_wave=1)
    assert [one.line_split(a) for a in (1, 2, 3)] == [(4, 64), (3, 64), (4, 40)]
    part = _init((256, 192, 160), bcs)  # 30720 lines on axis 1: two lines per wavefront
    assert [part.line_split(a) for a in (1, 2, 3)] == [(8, 32), (6, 32), (5, 32)]
    few = _init((256, 64, 100), bcs)  # axis 1 has 6400 lines: one line per wavefront
    assert [few.line_split(a) for a in (1, 2, 3)] == [(4, 64), (8, 8), (2, 50)]
    eight = _init((64, 64, 64, 64), ("periodic",) * 4)  # 262144 lines of 8 chunks of 8 rows
    assert [eight.line_split(a) for a in (1, 2, 3, 4)] == [(8, 8)] * 4
    assert eight.pass_kernel(1) == "k_first_pair<8, 64, 8, true, false, double>"
    assert eight.pass_kernel(3) == "k_mid_s<8, 2, 128, 8, true, double>"
    four = _init((64, 64, 64, 64), ("periodic",) * 4, lines_per_wave=4)  # 16 chunks of 4 rows
    assert [four.line_split(a) for a in (1, 2, 3, 4)] == [(4, 16)] * 4
    assert four.pass_kernel(3) == "k_mid_s<4, 2, 64, 4, true, double>"
    req = _init((256, 48, 10), bcs, lines_per_wave=4)  # four where n = 16 m, else two, else one
    assert [req.line_split(a) for a in (1, 2, 3)] == [(8, 32), (3, 16), (1, 10)]
    req.close()
    req8 = _init((256, 48, 10), bcs, lines_per_wave=8)  # eight where n = 8 m, else four, two, one
    assert [req8.line_split(a) for a in (1, 2, 3)] == [(8, 32), (6, 8), (1, 10)]
    req8.close()
    for p in (big, small, two, one, part, few, eight, four):
        p.close()
    with pytest.raises(etd.EtdError):
        _init((64, 64), ("periodic",) * 2, lines_per_wave=3)


def test_precision_option():
    from paper_2001_11220_amd import etd
    bcs = ("periodic", "neumann", "dirichlet")
    d64 = _init((256, 256, 160), bcs)
    f32 = _init((256, 256, 160), bcs, precision="f32")
    assert d64.pass_kernel(2) == "k_mid_s<8, 2, 32, 2, true, double>"
    # 2 x 10.5M floats = 84 MB per array: still above the non-temporal threshold
    assert f32.pass_kernel(2) == "k_mid_s<8, 2, 32, 2, true, float>"
    # the carried arrays halve; the FP64 tables are the same
    n = 256 * 256 * 160 * 2
    assert d64.ws_bytes - f32.ws_bytes == 6 * (8 - 4) * n
    small = _init((64, 48), ("neumann", "periodic"), precision="f32")  # 48 lines: two per wavefront
    assert small.pass_kernel(1) == "k_first_s<2, 2, 32, 2, false, false, float>"
    for p in (d64, f32, small):
        p.close()
    with pytest.raises(KeyError):
        _init((64, 64), ("periodic",) * 2, precision="f16")
    # the C ABI rejects unknown precision codes and a non-zero reserved field
    sch = etd.Scheme()
    for prec, res in ((3, 0), (0, 1)):
        sch.precision, sch.reserved = prec, res
        g = etd.Grid()
        g.d, g.s = 2, 2
        g.n[0], g.n[1] = 64, 64
        bc = (ctypes.c_int32 * 3)(1, 1, 0)
        D = (ctypes.c_double * 2)(0.1, 0.2)
        rx = etd.reaction_struct("brusselator", {"a": 1.0, "b": 3.0}, None, 2)
        ctx = ctypes.c_void_p()
        rc = etd.lib.etd_rdp_init(ctypes.byref(g), bc, D, 0.01, ctypes.byref(sch), ctypes.byref(rx),
                                  ctypes.byref(ctx))
        assert rc == etd.ETD_ERR_ARG


def test_complex_precision_option():
    from paper_2001_11220_amd import etd
    bcs = ("periodic",) * 3
    z = _init((200, 200, 200), bcs, D=(1 + 0.5j,), k=0.05, model="cgl_z", params={"beta": 1.3},
              h=(1.0, 1.0, 1.0), precision="c128")
    # chunk length 4: the streamed passes (16-line tiles, one line per wavefront)
    assert [z.pass_kernel(p) for p in (1, 2, 3)] == ["k_first_s<4, 1, 16, 1, true, false, zd>",
                                                     "k_mid_s<4, 1, 16, 1, true, zd>",
                                                     "k_last_s<4, 1, 16, 1, true, zd>"]
    assert z.line_split(1) == (4, 50)
    n = 200 ** 3
    assert z.ws_bytes >= 6 * 16 * n and z.ws_bytes < 6 * 16 * n + (1 << 20)
    small = _init((64, 48), ("neumann", "dirichlet"), D=(1j,), model="nls_z", params={"B": 0.0, "C": -1.0},
                  precision="c128")
    assert small.pass_kernel(2) == "k_last<1, 1, 8, false, zd>"
    # chunks of 5-8 rows: streamed passes with 8-line tiles
    long = _init((300, 448), ("periodic", "dirichlet"), D=(1 + 1j,), model="cgl_z", params={"beta": 1.0},
                 precision="c128")
    assert long.pass_kernel(1) == "k_first_s<5, 1, 8, 1, false, false, zd>"
    assert long.pass_kernel(2) == "k_last_s<7, 1, 8, 1, false, zd>"
    for p in (z, small, long):
        p.close()
    ok = dict(D=(1 + 1j,), model="cgl_z", params={"beta": 1.0}, precision="c128")
    cases = [
        ((1025, 16), ok, etd.ETD_ERR_UNSUPPORTED),  # longer than 64 chunks of 16 rows
        ((64, 16), dict(ok, lines_per_wave=2), etd.ETD_ERR_UNSUPPORTED),
        ((64, 16), dict(ok, D=(-0.1 + 1j,)), etd.ETD_ERR_ARG),  # Re D < 0
        ((64, 16), dict(ok, precision="f64", D=(1.0,)), etd.ETD_ERR_ARG),  # complex model, real context
        ((64, 16), dict(ok, model="cgl", D=(1.0, 1.0)), etd.ETD_ERR_ARG),  # real model, complex context
    ]
    for shape, kw, code in cases:
        with pytest.raises(etd.EtdError) as ei:
            _init(shape, ("periodic", "periodic"), **kw)
        assert ei.value.status == code, kw


def test_reaction_field_option():
    from paper_2001_11220_amd import etd
    kw = dict(D=(1j,), model="nls_z", params={"B": 0.0, "C": -1.0}, precision="c128")
    plain = _init((81, 81), ("neumann", "neumann"), **kw)
    etd_f = _lib().EtdRdp((81, 81), ("neumann", "neumann"), (1j,), 0.01, "nls_z", {"B": 0.0, "C": -1.0},
                          precision="c128", field=True)
    # two copies of the N-double field (each rounded up to 256 bytes)
    assert etd_f.ws_bytes - plain.ws_bytes == 2 * ((8 * 81 * 81 + 255) // 256 * 256)
    plain.close()
    etd_f.close()
    with pytest.raises(etd.EtdError) as ei:  # a field only for the Schroedinger model
        _lib().EtdRdp((64, 16), ("periodic",) * 2, (1 + 1j,), 0.01, "cgl_z", {"beta": 1.0}, precision="c128",
                      field=True)
    assert ei.value.status == etd.ETD_ERR_ARG


def test_four_dimensional_option():
    from paper_2001_11220_amd import etd
    e = _init((96, 8, 70, 5), ("neumann", "periodic", "dirichlet", "neumann"))
    assert [e.pass_kernel(p) for p in (1, 2, 3, 4)] == [
        "k_first<2, 2, 16, false, double>", "k_mid<1, 2, 16, false, double>",
        "k_mid<2, 2, 16, false, double>", "k_last<1, 2, 16, false, double>"]
    n1, n2, n3, n4 = 96, 8, 70, 5
    # layouts of the carried triples (axis strides 1..4): cyclic, pass p
    # writes axis p+1 fastest, then p+2, ..., 4, 1, ..., p
    assert e.layout(1)[1] == (n2 * n3 * n4, 1, n2, n2 * n3)
    assert e.layout(2)[1] == (n3 * n4, n3 * n4 * n1, 1, n3)
    assert e.layout(3)[1] == (n4, n4 * n1, n4 * n1 * n2, 1)
    assert e.layout(3)[0] == e.layout(1)[0]  # pass 3 writes the first triple again
    e.close()
    # the same layouts with a reaction field (its last-pass copy follows them)
    z = etd.EtdRdp((n1, n2, n3, n4), ("neumann", "periodic", "dirichlet", "neumann"), (1j,), 1e-3, "nls_z",
                   {"B": 0.4, "C": -1.0}, precision="c128", field=True)
    assert [z.layout(p)[1] for p in (1, 2, 3)] == [(n2 * n3 * n4, 1, n2, n2 * n3),
                                                   (n3 * n4, n3 * n4 * n1, 1, n3),
                                                   (n4, n4 * n1, n4 * n1 * n2, 1)]
    z.close()


def test_five_to_eight_dimensions_without_touching_the_gpu():
    """d = 5 .. 8 (Section 6's frame for any d): every pass reads its lines
    contiguously from a cyclic layout (pass p writes axis p+1 fastest, then
    p+2, ..., d, 1, ..., p), with the same kernels as the other dimensions;
    the reverse step is refused, single solves and a reaction field are
    accepted; the C ABI refuses d = 0 and d = 9."""
    from paper_2001_11220_amd import etd
    shape = (6, 5, 4, 3, 7)
    e = _init(shape, ("neumann", "periodic", "dirichlet", "neumann", "periodic"))
    assert len([e.pass_kernel(p) for p in range(1, 6)]) == 5
    N = int(np.prod(shape))
    for p in range(1, 5):
        order = [(p + i) % 5 for i in range(5)]  # fastest first
        want, st = [0] * 5, 1
        for a in order:
            want[a] = st
            st *= shape[a]
        assert e.layout(p)[1] == tuple(want), p
    assert e.layout(1)[0] == e.layout(3)[0] and e.layout(2)[0] == e.layout(4)[0] != e.layout(1)[0]
    assert e.adj_ws_bytes > 0
    u, x, g, ws = (ctypes.c_void_p(a) for a in (0x1000, 0x2000, 0x3000, 0x10000))
    assert etd.lib.etd_rdp_adjoint(e._ctx, u, x, g, g, ws, 1 << 40, None) == etd.ETD_ERR_UNSUPPORTED
    # single solves take any axis of any d; arguments are checked first
    assert etd.lib.etd_rdp_apply_solve(e._ctx, x, ws, e.ws_bytes, 6, 0, 3, None) == etd.ETD_ERR_ARG
    assert etd.lib.etd_rdp_apply_solve(e._ctx, x, ws, e.ws_bytes, 5, 0, 2, None) == etd.ETD_ERR_ARG
    e.close()
    e8 = _init((3,) * 8, ("periodic",) * 8, D=(0.3,), model="linear", params={"C": [[-0.5]]})
    assert e8.line_split(8) == (1, 3)
    e8.close()
    z = etd.EtdRdp((4,) * 5, ("periodic",) * 5, (1 + 1j,), 0.01, "nls_z", {"B": 1.0, "C": 1.0},
                   precision="c128", field=True)
    assert z.ws_bytes > 0
    z.close()
    with pytest.raises(ValueError):  # nine axes do not fit the grid struct
        _init((3,) * 9, ("periodic",) * 9)
    g = etd.Grid()  # the C ABI refuses d = 9 and d = 0
    for d in (9, 0):
        g.d, g.s = d, 2
        for i in range(etd.MAX_DIM):
            g.n[i] = 8
        bc = (ctypes.c_int32 * 9)(*([1] * 9))
        D = (ctypes.c_double * 2)(0.1, 0.2)
        rx = etd.reaction_struct("brusselator", {"a": 1.0, "b": 3.0}, None, 2)
        ctx = ctypes.c_void_p()
        rc = etd.lib.etd_rdp_init(ctypes.byref(g), bc, D, 0.01, None, ctypes.byref(rx), ctypes.byref(ctx))
        assert rc == etd.ETD_ERR_ARG


def test_one_dimensional_option():
    e = _init((512,), ("dirichlet",), D=(1.0, 10.0), k=1e-4, model="schnakenberg",
              params={"a": 0.1, "b": 0.9, "gamma": 1.0})
    # one pass: the last-pass kernel after an elementwise pre-pass
    assert e.pass_kernel(1) == "k_last_s<8, 2, 16, 1, false, double>"
    assert e.line_split(1) == (8, 64)
    e.close()


def test_tables_build_for_stiff_coefficients():
    # r = k D / h^2 up to ~5e6 still passes the residual self-check
    for D in (1e-9, 1.0, 1e3):
        p = _init((512, 64, 8), ("dirichlet", "periodic", "neumann"), D=(D, 10 * D), k=1.0)
        p.close()


def test_workspace_size_and_layout():
    p = _init((64, 32, 16), ("neumann", "periodic", "dirichlet"))
    N = 64 * 32 * 16
    arr = ((8 * N * 2 + 255) // 256) * 256
    (c1, c2, w), st1 = p.layout(1)
    assert c1 % 256 == 0 and c2 - c1 == arr and w - c2 == arr
    assert st1 == (32, 1, 64 * 32)  # [z][x][y]
    (d1, d2, dw), st2 = p.layout(2)
    assert d1 == w + arr and d2 - d1 == arr and dw - d2 == arr
    assert st2 == (32 * 16, 16, 1)  # [x][y][z]
    assert p.ws_bytes == dw + arr
    q = _init((64, 32), ("neumann", "periodic"))
    (e1, _, ew), st = q.layout(1)
    assert st == (32, 1) and q.ws_bytes == ew + ((8 * 64 * 32 * 2 + 255) // 256) * 256
    etd = _lib()
    with pytest.raises(etd.EtdError):
        q.layout(2)


def test_invalid_arguments():
    etd = _lib()
    E = etd.EtdError
    with pytest.raises(E) as e:
        _init((1,), ("neumann",), D=(0.2,), model="enzyme", params={})  # Neumann needs n >= 2
    assert e.value.status == etd.ETD_ERR_ARG
    for bad in [dict(k=0.0), dict(k=float("nan")), dict(D=(-1.0, 0.1)), dict(D=(float("inf"), 0.1)),
                dict(model="enzyme", params={}), dict(h=(-0.1, 0.0))]:
        with pytest.raises(E) as e:
            _init((8, 8), ("neumann", "neumann"), **bad)
        assert e.value.status == etd.ETD_ERR_ARG, bad
    with pytest.raises(E) as e:
        _init((2, 8), ("periodic", "neumann"))  # periodic needs n >= 3
    assert e.value.status == etd.ETD_ERR_ARG
    with pytest.raises(E) as e:
        _init((1, 8), ("neumann", "neumann"))  # Neumann needs n >= 2
    assert e.value.status == etd.ETD_ERR_ARG
    for n in (1025, 2048):
        with pytest.raises(E) as e:
            _init((n, 8), ("dirichlet", "neumann"))
        assert e.value.status == etd.ETD_ERR_UNSUPPORTED, n


def test_general_line_lengths_without_touching_the_gpu():
    """General line lengths (no split into <= 64 equal chunks of <= 8 rows)
    run the forward step with the general kernels, on any pass; the
    reverse-mode step, single solves and ensembles refuse them."""
    etd = _lib()
    p = _init((79, 1024, 361), ("dirichlet", "neumann", "periodic"), D=(0.5, 3.0), k=0.3)
    assert [p.line_split(a) for a in (1, 2, 3)] == [(2, 40), (16, 64), (6, 61)]
    assert [p.pass_kernel(a) for a in (1, 2, 3)] == ["kr_first<4, 2, 8, false, double>",
                                                     "kr_mid<16, 2, 8, double>",
                                                     "kr_last<8, 2, 8, double>"]
    u, ws = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x10000)
    x = ctypes.c_void_p(0x2000)
    assert etd.lib.etd_rdp_apply_solve(p._ctx, x, ws, p.ws_bytes, 1, 0, 3, None) == etd.ETD_ERR_UNSUPPORTED
    g = ctypes.c_void_p(0x3000)
    assert etd.lib.etd_rdp_adjoint(p._ctx, u, x, g, g, ws, 1 << 40, None) == etd.ETD_ERR_UNSUPPORTED
    p.close()
    z = _init((799, 16), ("periodic", "neumann"), D=(1 + 1j,), model="cgl_z", params={"beta": 1.0},
              precision="c128")
    assert z.pass_kernel(1) == "kr_first<16, 1, 4, false, zd>" and z.line_split(1) == (13, 62)
    z.close()
    f = _init((801, 16), ("neumann", "neumann"), precision="f32", scheme="etd1")
    assert f.pass_kernel(1) == "kr_first<16, 2, 8, true, float>" and f.line_split(1) == (13, 62)
    f.close()
    arr_t = (etd.Instance * 1)()
    arr_t[0].n[0], arr_t[0].n[1] = 79, 16
    arr_t[0].bc[0], arr_t[0].bc[1] = 1, 1
    arr_t[0].D[0] = 0.01
    ctx = ctypes.c_void_p()
    assert etd.lib.etd_rdp_batch_init(1, arr_t, 1, etd.MODELS["linear"], 0.01, None,
                                      ctypes.byref(ctx)) == etd.ETD_ERR_UNSUPPORTED


def test_null_pointers_rejected():
    etd = _lib()
    out = ctypes.c_void_p()
    assert etd.lib.etd_rdp_init(None, None, None, 0.1, None, None, ctypes.byref(out)) == etd.ETD_ERR_ARG
    nb = ctypes.c_size_t()
    assert etd.lib.etd_rdp_workspace_bytes(None, ctypes.byref(nb)) == etd.ETD_ERR_ARG
    assert etd.lib.etd_rdp_step(None, None, None, 0, 1, None) == etd.ETD_ERR_ARG
    assert etd.lib.etd_rdp_destroy(None) == etd.ETD_OK


def test_step_validates_workspace_without_touching_the_gpu():
    etd = _lib()
    p = _init((16, 16), ("neumann", "neumann"))
    ctx = p._ctx
    fake_u = ctypes.c_void_p(0x1000)
    # NULL, misaligned, too small: all rejected before any HIP call
    assert etd.lib.etd_rdp_step(ctx, fake_u, None, p.ws_bytes, 1, None) == etd.ETD_ERR_WORKSPACE
    assert etd.lib.etd_rdp_step(ctx, fake_u, ctypes.c_void_p(0x1008), p.ws_bytes, 1, None) == etd.ETD_ERR_WORKSPACE
    assert etd.lib.etd_rdp_step(ctx, fake_u, ctypes.c_void_p(0x2000), p.ws_bytes - 8, 1, None) == etd.ETD_ERR_WORKSPACE
    assert etd.lib.etd_rdp_step(ctx, fake_u, ctypes.c_void_p(0x2000), p.ws_bytes, -1, None) == etd.ETD_ERR_ARG
    assert etd.lib.etd_rdp_apply_solve(ctx, fake_u, ctypes.c_void_p(0x2000), p.ws_bytes, 1, 0, 2, None) == etd.ETD_ERR_ARG
    assert etd.lib.etd_rdp_apply_solve(ctx, fake_u, ctypes.c_void_p(0x2000), p.ws_bytes, 3, 0, 1, None) == etd.ETD_ERR_ARG
    assert etd.status_string(etd.ETD_ERR_WORKSPACE).startswith("workspace")
    # zero steps: a no-op that enqueues nothing (valid arguments, no HIP call)
    assert etd.lib.etd_rdp_step(ctx, fake_u, ctypes.c_void_p(0x2000), p.ws_bytes, 0, None) == etd.ETD_OK


def test_empty_and_degenerate_grids():
    etd = _lib()
    for shape, bcs in (((0, 8), ("dirichlet", "neumann")),      # an empty axis
                       ((8, 1), ("neumann", "neumann")),        # Neumann needs two points
                       ((8, 2), ("periodic", "periodic"))):     # periodic needs three
        with pytest.raises(etd.EtdError) as ei:
            _init(shape, bcs)
        assert ei.value.status == etd.ETD_ERR_ARG, shape
    one = _init((1, 1), ("dirichlet", "dirichlet"))  # a single cell is a valid problem
    assert one.line_split(1) == (1, 1) and one.line_split(2) == (1, 1)
    one.close()


def test_adjoint_workspace_and_gradient_size():
    N = 64 * 32 * 16
    arr = ((8 * N * 2 + 255) // 256) * 256
    p = _init((64, 32, 16), ("neumann", "periodic", "dirichlet"))
    (c1, _, _), _ = p.layout(1)
    # tables, nine carried arrays (3-D), block sums; the forward layout is a prefix
    assert p.adj_ws_bytes > c1 + 9 * arr and p.adj_ws_bytes >= p.ws_bytes
    q = _init((64, 32), ("neumann", "periodic"))
    arr2 = ((8 * 64 * 32 * 2 + 255) // 256) * 256
    assert q.adj_ws_bytes > q.layout(1)[0][0] + 6 * arr2
    sizes = {"brusselator": ({"a": 1.0, "b": 3.0}, 2, 4), "gray_scott": ({"F": 0.04, "kappa": 0.06}, 2, 4),
             "schnakenberg": ({"a": 0.1, "b": 0.9, "gamma": 1.0}, 2, 5), "cgl": ({"beta": 0.5}, 2, 3),
             "linear": ({"C": [[0.1, 0.2], [0.3, 0.4]]}, 2, 6), "enzyme": ({}, 1, 1)}
    for model, (params, s, n) in sizes.items():
        D = (0.1, 0.2)[:s]
        e = _init((16, 16), ("neumann", "neumann"), D=D, model=model, params=params)
        assert e.grad_size == n, model
        assert len(e.param_vector()) == n
        assert e.param_vector()[:s] == list(D)
    e = _init((16, 16), ("neumann", "neumann"), D=(0.3,), model="linear", params={"C": [[-0.5]]})
    assert e.grad_size == 2 and e.param_vector() == [0.3, -0.5]


def test_adjoint_validates_arguments_without_touching_the_gpu():
    etd = _lib()
    p = _init((16, 16), ("neumann", "neumann"))
    ctx = p._ctx
    u, lam, lo, g = (ctypes.c_void_p(a) for a in (0x1000, 0x2000, 0x3000, 0x4000))
    ws = ctypes.c_void_p(0x10000)
    f = etd.lib.etd_rdp_adjoint
    assert f(None, u, lam, lo, g, ws, p.adj_ws_bytes, None) == etd.ETD_ERR_ARG
    assert f(ctx, None, lam, lo, g, ws, p.adj_ws_bytes, None) == etd.ETD_ERR_ARG
    assert f(ctx, u, None, lo, g, ws, p.adj_ws_bytes, None) == etd.ETD_ERR_ARG
    assert f(ctx, u, lam, None, g, ws, p.adj_ws_bytes, None) == etd.ETD_ERR_ARG
    assert f(ctx, u, lam, lo, None, ws, p.adj_ws_bytes, None) == etd.ETD_ERR_ARG
    assert f(ctx, u, lam, u, g, ws, p.adj_ws_bytes, None) == etd.ETD_ERR_ARG  # lam_n == u_n
    assert f(ctx, u, lam, lo, g, None, p.adj_ws_bytes, None) == etd.ETD_ERR_WORKSPACE
    assert f(ctx, u, lam, lo, g, ctypes.c_void_p(0x10008), p.adj_ws_bytes, None) == etd.ETD_ERR_WORKSPACE
    # the forward workspace is too small for the reverse step
    assert f(ctx, u, lam, lo, g, ws, p.ws_bytes, None) == etd.ETD_ERR_WORKSPACE
    q = _init((16, 16), ("neumann", "neumann"), scheme="etd1")
    assert f(q._ctx, u, lam, lo, g, ws, q.adj_ws_bytes, None) == etd.ETD_ERR_UNSUPPORTED
    n = ctypes.c_int32()
    assert etd.lib.etd_rdp_grad_size(None, ctypes.byref(n)) == etd.ETD_ERR_ARG


def test_kept_steps_validate_arguments_without_touching_the_gpu():
    """etd_rdp_keep_bytes sizes one step's kept arrays (3 triples' worth in
    2-D, 6 in 3-D, each array rounded up to 256 bytes) and is refused where
    the reverse step is; the kept step and kept reverse step refuse missing,
    small and misaligned buffers before any device work."""
    etd = _lib()
    nb = ctypes.c_size_t()
    p = _init((16, 16), ("neumann", "neumann"))
    assert etd.lib.etd_rdp_keep_bytes(p._ctx, ctypes.byref(nb)) == etd.ETD_OK
    assert nb.value == 3 * 2 * 16 * 16 * 8
    assert etd.lib.etd_rdp_keep_bytes(None, ctypes.byref(nb)) == etd.ETD_ERR_ARG
    assert etd.lib.etd_rdp_keep_bytes(p._ctx, None) == etd.ETD_ERR_ARG
    q = _init((10, 6, 5), ("neumann", "periodic", "dirichlet"), D=(0.3,), model="linear", params={"C": [[-0.5]]})
    assert etd.lib.etd_rdp_keep_bytes(q._ctx, ctypes.byref(nb)) == etd.ETD_OK
    assert nb.value == 6 * 2560  # 300 doubles = 2400 bytes, rounded up to 2560
    q.close()
    for kw in (dict(scheme="etd1"), dict(precision="f32")):
        r = _init((16, 16), ("neumann", "neumann"), **kw)
        assert etd.lib.etd_rdp_keep_bytes(r._ctx, ctypes.byref(nb)) == etd.ETD_ERR_UNSUPPORTED, kw
        r.close()
    for shape, bcs in (((79, 16), ("dirichlet", "neumann")), ((8,), ("neumann",)),
                       ((4, 4, 4, 4), ("neumann",) * 4)):
        r = _init(shape, bcs)
        assert etd.lib.etd_rdp_keep_bytes(r._ctx, ctypes.byref(nb)) == etd.ETD_ERR_UNSUPPORTED, shape
        r.close()
    need = 3 * 2 * 16 * 16 * 8
    u, lam, lo, g = (ctypes.c_void_p(a) for a in (0x1000, 0x2000, 0x3000, 0x4000))
    ws, kp = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x100000)
    sk, ak = etd.lib.etd_rdp_step_keep, etd.lib.etd_rdp_adjoint_kept
    assert sk(p._ctx, u, u, ws, p.ws_bytes, None, need, None) == etd.ETD_ERR_ARG
    assert sk(p._ctx, u, u, ws, p.ws_bytes, kp, need - 8, None) == etd.ETD_ERR_ARG
    assert sk(p._ctx, u, u, ws, p.ws_bytes, ctypes.c_void_p(0x100008), need, None) == etd.ETD_ERR_ARG
    assert sk(p._ctx, None, u, ws, p.ws_bytes, kp, need, None) == etd.ETD_ERR_ARG
    assert sk(p._ctx, u, None, ws, p.ws_bytes, kp, need, None) == etd.ETD_ERR_ARG
    # distinct states that overlap (the state is 2 * 16 * 16 doubles = 4096 bytes)
    assert sk(p._ctx, u, ctypes.c_void_p(0x1000 + 4088), ws, p.ws_bytes, kp, need, None) == etd.ETD_ERR_ARG
    assert sk(p._ctx, ctypes.c_void_p(0x1000 + 4088), u, ws, p.ws_bytes, kp, need, None) == etd.ETD_ERR_ARG
    assert sk(p._ctx, u, u, None, p.ws_bytes, kp, need, None) == etd.ETD_ERR_WORKSPACE
    assert sk(p._ctx, u, ctypes.c_void_p(0x1000 + 4096), None, p.ws_bytes, kp, need, None) == etd.ETD_ERR_WORKSPACE
    assert ak(p._ctx, u, None, need, lam, lo, g, ws, p.adj_ws_bytes, None) == etd.ETD_ERR_ARG
    assert ak(p._ctx, u, kp, need - 8, lam, lo, g, ws, p.adj_ws_bytes, None) == etd.ETD_ERR_ARG
    assert ak(p._ctx, u, ctypes.c_void_p(0x100008), need, lam, lo, g, ws, p.adj_ws_bytes, None) == etd.ETD_ERR_ARG
    assert ak(p._ctx, u, kp, need, lam, u, g, ws, p.adj_ws_bytes, None) == etd.ETD_ERR_ARG  # lam_n == u_n
    assert ak(p._ctx, u, kp, need, lam, lo, g, ws, p.ws_bytes, None) == etd.ETD_ERR_WORKSPACE
    p.close()


def test_calibration_sweeps_validate_arguments_without_touching_the_gpu():
    etd = _lib()
    f = etd.lib.etd_calib_stream
    a, b = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert f(6, a, b, 4096, 8, None) == etd.ETD_ERR_ARG       # unknown kind
    assert f(-1, a, b, 4096, 8, None) == etd.ETD_ERR_ARG
    for kind in (0, 1, 3, 5):
        assert f(kind, None, b, 4096, 8, None) == etd.ETD_ERR_ARG  # needs a source
    for kind in range(6):
        assert f(kind, a, None, 4096, 8, None) == etd.ETD_ERR_ARG
        assert f(kind, a, b, 4100, 8, None) == etd.ETD_ERR_ARG     # not whole 16-byte elements
        assert f(kind, a, ctypes.c_void_p(0x2008), 4096, 8, None) == etd.ETD_ERR_ARG
        assert f(kind, a, b, 4096, 0, None) == etd.ETD_ERR_ARG
        assert f(kind, a, b, 0, 8, None) == etd.ETD_OK             # nothing to do


def test_batch_precision_option_without_touching_the_gpu():
    """An FP32 ensemble halves the carried arrays; each step entry point
    refuses the other precision before any device work."""
    etd = _lib()
    ins = [dict(shape=(40, 24), bcs=("neumann", "periodic"), D=(0.02, 0.01), params={"a": 1.0, "b": 3.0}),
           dict(shape=(17, 64), bcs=("periodic", "dirichlet"), D=(0.01, 0.03), params={"a": 1.2, "b": 2.8})]
    b64 = etd.EtdRdpBatch(ins, 2, "brusselator", 0.01)
    b32 = etd.EtdRdpBatch(ins, 2, "brusselator", 0.01, precision="f32")
    assert b32.offsets == b64.offsets and b32.launches_per_step == b64.launches_per_step
    # the three carried arrays (each rounded up to 256 bytes) are the only
    # part of the workspace that depends on the element size
    ru = lambda v: (v + 255) // 256 * 256  # noqa: E731
    tot = b64.offsets[-1]
    assert b64.ws_bytes - b32.ws_bytes == 3 * (ru(8 * tot) - ru(4 * tot))
    u, ws = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x10000)
    assert etd.lib.etd_rdp_batch_step(b32._ctx, u, ws, b32.ws_bytes, 1, 0, None) == etd.ETD_ERR_ARG
    assert etd.lib.etd_rdp_batch_step_f32(b64._ctx, u, ws, b64.ws_bytes, 1, 0, None) == etd.ETD_ERR_ARG
    assert etd.lib.etd_rdp_batch_step_f32(None, u, ws, b64.ws_bytes, 1, 0, None) == etd.ETD_ERR_ARG
    assert etd.lib.etd_rdp_batch_step_f32(b32._ctx, u, None, b32.ws_bytes, 1, 0, None) == etd.ETD_ERR_WORKSPACE
    # zero steps is a no-op that touches nothing
    assert etd.lib.etd_rdp_batch_step_f32(b32._ctx, u, ws, b32.ws_bytes, 0, 0, None) == etd.ETD_OK
    with pytest.raises(ValueError):
        etd.EtdRdpBatch(ins, 2, "brusselator", 0.01, precision="c128")
    sch = etd.Scheme()
    sch.precision = etd.PRECISIONS["c128"]
    arr_t = (etd.Instance * 1)()
    arr_t[0].n[0], arr_t[0].n[1] = 16, 16
    arr_t[0].bc[0], arr_t[0].bc[1] = 1, 1
    arr_t[0].D[0] = 0.01
    ctx = ctypes.c_void_p()
    assert etd.lib.etd_rdp_batch_init(1, arr_t, 1, etd.MODELS["linear"], 0.01, ctypes.byref(sch),
                                      ctypes.byref(ctx)) == etd.ETD_ERR_UNSUPPORTED


def test_batch_groups_and_plans_without_touching_the_gpu():
    """Instances of one grid shape form a group stored at equal spacing; the
    default plan and set_plan only take forms a (group, pass) allows."""
    etd = _lib()
    ins = [dict(shape=(64, 64), bcs=("neumann", "periodic"), D=(0.02, 0.01), params={"a": 1.0, "b": 3.0}),
           dict(shape=(40, 30), bcs=("periodic", "dirichlet"), D=(0.01, 0.03), params={"a": 1.0, "b": 2.0}),
           dict(shape=(64, 64), bcs=("dirichlet", "neumann"), D=(0.03, 0.02), params={"a": 1.0, "b": 3.5}),
           dict(shape=(512, 40), bcs=("neumann", "neumann"), D=(0.01, 0.01), params={"a": 1.0, "b": 2.5})]
    b = etd.EtdRdpBatch(ins, 2, "brusselator", 0.01)
    assert b.groups() == [(64, 64, 2), (40, 30, 1), (512, 40, 1)]
    assert b.launches_per_step == 6
    off = b.offsets
    assert off[2] - off[0] == 2 * 64 * 64  # the two 64^2 instances, back to back
    assert off[-1] == 2 * (2 * 64 * 64) + 2 * 40 * 30 + 2 * 512 * 40
    assert all(v % 32 == 0 for v in off)
    # lines of 64 = 32 x 2: every form; 40 and 30 (chunks of 1): unsplit only;
    # 512 (chunks of 8) on axis 1: unsplit or streamed
    allowed = {(g, p): [f for f in range(3) if b.form_allowed(g, p, f)] for g in range(3) for p in range(2)}
    assert allowed[(0, 0)] == [0, 2] and allowed[(0, 1)] == [0, 2]   # 64 = 32 x 2 (m1 = 1)
    assert allowed[(1, 0)] == [0] and allowed[(1, 1)] == [0]
    assert allowed[(2, 0)] == [0, 1] and allowed[(2, 1)] == [0]
    assert b.plan == [0, 0, 0, 0, 1, 0]
    b.plan = [2, 2, 0, 0, 0, 0]
    assert b.plan == [2, 2, 0, 0, 0, 0]
    with pytest.raises(etd.EtdError):
        b.plan = [1, 0, 0, 0, 0, 0]  # 64: chunks of one row, no streamed form
    assert b.plan == [2, 2, 0, 0, 0, 0]
    e1 = etd.EtdRdpBatch(ins, 2, "brusselator", 0.01, scheme="etd1")
    assert not e1.form_allowed(2, 0, 1) and not e1.form_allowed(0, 0, 2) and e1.form_allowed(0, 1, 2)
    b.close()
    e1.close()
