"""Host-side checks of the C ABI (no GPU): the library loads, exports every
declared entry point, and its pure-host calls validate parameters."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(vbgs_[a-z0-9_]+)\s*\(", txt))
    return names


def _lib():
    from paper_2603_08499_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libvbgs.so not built")
    return L.load(), L


def test_every_declared_symbol_is_exported():
    lib, _ = _lib()
    declared = _declared()
    assert {"vbgs_init", "vbgs_estep_stats", "vbgs_update", "vbgs_elbo"} <= declared
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing


def test_query_sizes_and_validation():
    import paper_2603_08499_amd as P
    _lib()
    p = P.make_params(6, 100000, 307200)
    sb, wb = P.query_sizes(p)
    assert sb == 256 + 2 * 100000 * 48 * 8
    assert wb > 307200 * 32 * 8 and wb % 256 == 0
    bad = [dict(D=0), dict(D=9), dict(K=0), dict(n_max=-1)]
    for b in bad:
        args = dict(D=6, K=10, n_max=10)
        args.update(b)
        with pytest.raises(P.VBGSError):
            P.query_sizes(P.make_params(**args))
    with pytest.raises(P.VBGSError) as e:
        P.query_sizes(P.make_params(7, 10, 10, score_prec="bf16"))
    assert e.value.status == -7
    p = P.make_params(7, 10, 10, score_prec="fp64")
    P.query_sizes(p)
    p = P.make_params(6, 10, 10, nu0=4.0)
    with pytest.raises(P.VBGSError):
        P.query_sizes(p)
    # the proposal needs the exact MFMA mode; its weights and Adam moments live in the state
    with pytest.raises(P.VBGSError):
        P.query_sizes(P.make_params(6, 10, 10, score_prec="fp64", proposal=True))
    # the automatic screen precision belongs to the exact mode without the proposal
    P.query_sizes(P.make_params(6, 10, 10, score_prec="auto"))
    for args in (dict(exact=False), dict(proposal=True)):
        with pytest.raises(P.VBGSError) as e:
            P.query_sizes(P.make_params(6, 10, 10, score_prec="auto", **args))
        assert e.value.status == -7
    # the FP8 tier is a plain tier: the exact mode and the proposal reject it
    P.query_sizes(P.make_params(6, 10, 10, score_prec="fp8", exact=False))
    for args in (dict(exact=True), dict(exact=True, proposal=True)):
        with pytest.raises(P.VBGSError) as e:
            P.query_sizes(P.make_params(6, 10, 10, score_prec="fp8", **args))
        assert e.value.status == -7
    with pytest.raises(P.VBGSError) as e:
        P.query_sizes(P.make_params(7, 10, 10, score_prec="fp8", exact=False))
    assert e.value.status == -7
    # culling coordinates: 0 (automatic) or 1..min(D, 3)
    P.query_sizes(P.make_params(5, 10, 10, cull_dims=2))
    for args in (dict(D=6, cull_dims=4), dict(D=2, cull_dims=3), dict(D=6, cull_dims=-1)):
        with pytest.raises(P.VBGSError):
            P.query_sizes(P.make_params(K=10, n_max=10, **args))
    # two-factor model: split inside 0..D-1, room in the record for the second kappa, nu, no proposal
    P.query_sizes(P.make_params(6, 10, 10, modal_split=3))
    P.query_sizes(P.make_params(7, 10, 10, score_prec="fp64", modal_split=3))
    for args, status in [(dict(D=6, modal_split=6), -1), (dict(D=6, modal_split=-1), -1),
                         (dict(D=8, score_prec="fp64", modal_split=3), -7),
                         (dict(D=6, modal_split=3, proposal=True), -7)]:
        with pytest.raises(P.VBGSError) as e:
            P.query_sizes(P.make_params(K=10, n_max=10, **args))
        assert e.value.status == status, args
    s0, w0 = P.query_sizes(P.make_params(6, 1000, 500))
    s1, w1 = P.query_sizes(P.make_params(6, 1000, 500, proposal=True))
    n_train = 128 * 6 + 128 + 128 * 128 + 128 + 1000 * 128 + 1000
    assert s1 - s0 >= 3 * n_train * 4 and w1 > w0


def test_params_struct_layout_matches_header():
    from paper_2603_08499_amd import _lib as L
    P = L.Params
    assert ctypes.sizeof(P) == 120
    assert P.screen_margin.offset == 56 and P.n_split.offset == 64 and P.proposal.offset == 68
    assert P.C.offset == 72 and P.train_batch.offset == 76 and P.cull.offset == 80
    assert P.modal_split.offset == 84 and P.cull_dims.offset == 88 and P.reserved.offset == 96
    # the same offsets as the C compiler gives the header's struct
    import os
    import subprocess
    import tempfile
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    names = [n for n, _ in P._fields_]
    src = "#include <stdio.h>\n#include \"vbgs.h\"\nint main(void) {\n printf(\"%zu\\n\", sizeof(vbgs_params));\n"
    src += "".join(' printf("%%zu\\n", offsetof(vbgs_params, %s));\n' % n for n in names) + " return 0;\n}\n"
    with tempfile.TemporaryDirectory() as d:
        with open(os.path.join(d, "o.c"), "w") as f:
            f.write(src)
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(root, "include"), "-o", os.path.join(d, "o"),
                               os.path.join(d, "o.c")])
        got = [int(v) for v in subprocess.check_output([os.path.join(d, "o")]).split()]
    assert got == [ctypes.sizeof(P)] + [getattr(P, n).offset for n in names]


def test_null_context_calls_fail_cleanly():
    lib, L = _lib()
    assert lib.vbgs_estep_stats(None, None, 0, None, None, None) == -1
    assert lib.vbgs_update(None, 0, None) == -1
    assert lib.vbgs_elbo(None, None, 0, None, None) == -1
    assert lib.vbgs_last_error(None) == b"null context"
    lib.vbgs_destroy(None)
