"""The C-ABI library loads and exports every entry point of include/ibdns.h;
host-side argument validation (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ibdns.h")).read()
    return sorted(set(re.findall(r"\b(ibdns_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    import paper_2103_08246_amd as ib
    assert sorted(ib.EXPORTED) == declared_symbols()


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2103_08246_amd", "libibdns.so"))
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_workspace_size_validation():
    import paper_2103_08246_amd as ib
    good = ib.make_domain(64, 32, 32, 4.0, 2.0, 2.0, 200.0, dt=1e-3)
    n = ib.workspace_size(good, 0, 16)
    P = 80  # pitch of nx+1 = 65 rounded to 16
    assert n > 11 * P * 32 * 32 * 8
    bad = [ib.make_domain(64, 30, 32, 4.0, 1.875, 2.0, 200.0, dt=1e-3),   # 30 = 2*3*5
           ib.make_domain(64, 32, 32, 4.0, 2.5, 2.0, 200.0, dt=1e-3),     # anisotropic h
           ib.make_domain(4, 32, 32, 0.25, 2.0, 2.0, 200.0, dt=1e-3),     # nx too small
           ib.make_domain(64, 32, 32, 4.0, 2.0, 2.0, 200.0, dt=0.0, cfl=1.5),
           ib.make_domain(64, 32, 32, 4.0, 2.0, 2.0, 200.0, dt=1e-3, precision=7)]
    # mixed precision pads rows to 32 elements (FP32 rows on 128-byte lines): 96, not 80
    m = ib.workspace_size(ib.make_domain(64, 32, 32, 4.0, 2.0, 2.0, 200.0, dt=1e-3,
                                         precision=ib.MIXED), 0, 16)
    assert m > 11 * 96 * 32 * 32 * 8 and m > n
    for d in bad:
        with pytest.raises(ib.IbdnsError) as e:
            ib.workspace_size(d)
        assert e.value.code == ib.EINVAL


def test_strerror():
    import paper_2103_08246_amd as ib
    assert "workspace" in ib.strerror(ib.ENOMEM)
    assert ib.strerror(ib.OK) == "ok"


def test_probe_workspace_size():
    import paper_2103_08246_amd as ib
    lib = ib.lib()
    out = ctypes.c_size_t(0)
    assert lib.ibdns_probe_workspace_size(3, 5, ctypes.byref(out)) == ib.OK
    n = 27
    up = lambda b: (b + 255) // 256 * 256   # noqa: E731  (256-byte carving)
    assert out.value == up(3 * n * 8) + up(n * (10 + 2 * 5) * 8) + up(n * 2 * 5 * 8)
    for n_x, n_lags in ((0, 5), (3, 0), (3, 4097)):
        assert lib.ibdns_probe_workspace_size(n_x, n_lags, ctypes.byref(out)) == ib.EINVAL


def test_diffusion_mode_validation():
    import paper_2103_08246_amd as ib
    out = ctypes.c_size_t(0)
    lib = ib.lib()
    cn = ib.make_domain(64, 32, 32, 4.0, 2.0, 2.0, 200.0, dt=1e-3, diffusion=ib.DIFFUSION_CN)
    assert lib.ibdns_workspace_size(ctypes.byref(cn), 0, 0, ctypes.byref(out)) == ib.OK
    cn_mixed = ib.make_domain(64, 32, 32, 4.0, 2.0, 2.0, 200.0, dt=1e-3, precision=ib.MIXED,
                              diffusion=ib.DIFFUSION_CN)
    assert lib.ibdns_workspace_size(ctypes.byref(cn_mixed), 0, 0, ctypes.byref(out)) == ib.OK
    bad = ib.make_domain(64, 32, 32, 4.0, 2.0, 2.0, 200.0, dt=1e-3, diffusion=2)
    assert lib.ibdns_workspace_size(ctypes.byref(bad), 0, 0, ctypes.byref(out)) == ib.EINVAL
