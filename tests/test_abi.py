"""The C-ABI library loads and exports every entry point its header declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_symbols():
    syms = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(spdz_\w+)\s*\(", text, flags=re.M):
            syms.add(m.group(1))
    return syms


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ["spdz_ctx_create", "spdz_ctx_destroy", "spdz_open", "spdz_mul_batch", "spdz_linear",
              "spdz_reduce_add", "spdz_mul_fused", "spdz_mac_check", "spdz_status_str"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2512_11112_amd import spdz
    lib = spdz.lib()
    missing = [s for s in sorted(declared_symbols()) if not hasattr(lib, s)]
    assert not missing, missing


def test_status_strings_and_host_only_errors():
    from paper_2512_11112_amd import spdz
    assert spdz.status_str(0) == "ok"
    assert "MAC" in spdz.status_str(1)
    # modulus and party-count validation happen before any device call
    lib = spdz.lib()
    h = ctypes.c_void_p()
    al = (ctypes.c_uint64 * 2)(1, 2)
    bad_p = spdz.limbs((1 << 31) - 1, 1)
    assert lib.spdz_ctx_create(ctypes.byref(h), 2, bad_p, 1, al, 0, None) == -2
    assert lib.spdz_ctx_create(ctypes.byref(h), 9, spdz.limbs(spdz.P61, 1), 1, al, 0, None) == -7
    assert lib.spdz_ctx_create(ctypes.byref(h), 1, spdz.limbs(spdz.P61, 1), 1, al, 0, None) == -7
    # non-canonical alpha share is rejected before any device call
    al_bad = (ctypes.c_uint64 * 2)(spdz.P61, 0)
    assert lib.spdz_ctx_create(ctypes.byref(h), 2, spdz.limbs(spdz.P61, 1), 1, al_bad, 0, None) == -1
    assert lib.spdz_ctx_destroy(None) == 0


@pytest.mark.parametrize("p", [(1 << 61) - 1, (1 << 127) - 1])
def test_host_alpha_dealer_matches_oracle(p):
    from paper_2512_11112_amd import spdz
    import oracle.ref as R
    for seed in (0, 1, 12345):
        assert spdz.deal_alpha(p, 5, seed) == R.alpha_shares(p, 5, seed)
