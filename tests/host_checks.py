"""Host-logic checks of the C-ABI library that need no GPU, run as a script
in a child process against the host-sanitized variant (librbfl_san.so,
AddressSanitizer + UndefinedBehaviorSanitizer on the host pass) with the
clang ASan runtime preloaded.  Everything here returns before the first
device call: spec validation of rbfl_build, argument checks of the entry
points, store-file parsing of rbfl_load (including damaged files), and the
host-only variant counts.  Any sanitizer report aborts the process with a
non-zero status; a wrong return code raises.

Usage: python tests/host_checks.py <library path>
"""
import ctypes as C
import os
import struct
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2508_04172_amd import rbfl  # noqa: E402  (binding types only; no library load, no torch)
from paper_2508_04172_amd import workloads as wl  # noqa: E402


def with_checksum(body: bytes) -> bytes:
    """body followed by its FNV-1a hash over 8-byte little-endian words (a
    short last word zero-padded), the layout rbfl_save writes."""
    h = 0xcbf29ce484222325
    for i in range(0, len(body), 8):
        h = ((h ^ int.from_bytes(body[i:i + 8], "little")) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return bytes(body) + struct.pack("<Q", h)


def store_file(sections, fmt=1, abi=rbfl.ABI_VERSION, magic=b"RBFLSTOR"):
    """A store file with a valid checksum around the given raw sections."""
    body = bytearray(magic + struct.pack("<IIQ", fmt, abi, len(sections)))
    for tag, esize, payload in sections:
        body += struct.pack("<IIQ", tag, esize, len(payload) // esize) + payload
        body += bytes((8 - len(payload) % 8) % 8)
    return with_checksum(bytes(body))


def main(path):
    lib = C.CDLL(path)
    lib.rbfl_last_error.restype = C.c_char_p
    lib.rbfl_build.argtypes = [C.POINTER(rbfl.BuildSpec), C.c_void_p, C.POINTER(C.c_void_p)]
    lib.rbfl_load.argtypes = [C.c_char_p, C.c_void_p, C.POINTER(C.c_void_p)]
    n_checks = 0

    def expect(code, want, what):
        nonlocal n_checks
        n_checks += 1
        if code != want:
            raise AssertionError(f"{what}: returned {code}, expected {want} ({lib.rbfl_last_error()!r})")
        if want != rbfl.OK and not lib.rbfl_last_error():
            raise AssertionError(f"{what}: no error message")

    # ---- spec validation: one field broken at a time
    cfg = wl.SMALL_BANDED
    keep = []
    inj = wl.injection_extrinsics(cfg)

    def spec():
        return rbfl.spec_from_config(cfg, None, inj, None, keep)

    nan = float("nan")
    bad_geom = np.array(cfg.sites, dtype=np.float64)
    bad_geom[1, 2] = nan
    keep.append(bad_geom)
    n_f = int(round(cfg.fs * cfg.seg_len)) // 2 + 1
    bad_psd = np.ones((cfg.n_det, n_f))
    bad_psd[2, 100] = -1.0
    keep.append(bad_psd)
    breaks = {
        "abi": lambda s: setattr(s, "abi_version", rbfl.ABI_VERSION + 1),
        "n_det 0": lambda s: setattr(s, "n_det", 0),
        "n_det 5": lambda s: setattr(s, "n_det", 5),
        "n_modes 0": lambda s: setattr(s, "n_modes", 0),
        "n_modes 6": lambda s: setattr(s, "n_modes", 6),
        "mode (3,1)": lambda s: (s.modes[1].__setitem__(0, 3), s.modes[1].__setitem__(1, 1)),
        "duplicate mode": lambda s: (s.modes[1].__setitem__(0, 2), s.modes[1].__setitem__(1, 2)),
        "fs": lambda s: setattr(s, "fs", -1.0),
        "odd samples": lambda s: setattr(s, "seg_len", 8.0 + 1.0 / cfg.fs),
        "f_low": lambda s: setattr(s, "f_low", cfg.fs),
        "det_geom NULL": lambda s: setattr(s, "det_geom", C.POINTER(C.c_double)()),
        "det_geom NaN": lambda s: setattr(s, "det_geom", bad_geom.ctypes.data_as(C.POINTER(C.c_double))),
        "psd_scale": lambda s: setattr(s, "psd_scale", 0.0),
        "psd negative": lambda s: setattr(s, "psd", bad_psd.ctypes.data_as(C.POINTER(C.c_double))),
        "inj_snr": lambda s: setattr(s, "inj_snr", 0.0),
        "inj masses": lambda s: (s.inj_phys.__setitem__(0, 1.0), s.inj_phys.__setitem__(1, 2.0)),
        "centre masses": lambda s: s.center_phys.__setitem__(1, 9.0),
        "centre spin": lambda s: s.center_phys.__setitem__(2, 1.5),
        "match 0": lambda s: setattr(s, "match", 0.0),
        "match 1": lambda s: setattr(s, "match", 1.0),
        "t_trig off grid": lambda s: setattr(s, "t_trig", cfg.t_trig + 0.3 / cfg.fs),
        "t_trig outside": lambda s: setattr(s, "t_trig", cfg.seg_len + 1.0),
        "half_window": lambda s: setattr(s, "half_window", 1.0 / cfg.fs),
        "poly_degree": lambda s: setattr(s, "poly_degree", 4),
        "n_nodes": lambda s: setattr(s, "n_nodes", 5),
        "q 0": lambda s: setattr(s, "q", 0),
        "q > N": lambda s: setattr(s, "q", cfg.n_nodes + 1),
        "eps": lambda s: setattr(s, "eps", -1.0),
        "chi_max": lambda s: setattr(s, "chi_max", 0.0),
        "flags": lambda s: setattr(s, "flags", 0x80),
        "f_ref": lambda s: setattr(s, "f_ref", cfg.fs),
        "earth_rate": lambda s: setattr(s, "earth_rate", nan),
        "n_bands": lambda s: setattr(s, "n_bands", rbfl.MAX_BANDS + 1),
        "n_bands negative": lambda s: setattr(s, "n_bands", -1),
    }
    for label, brk in breaks.items():
        s = spec()
        brk(s)
        h = C.c_void_p()
        expect(lib.rbfl_build(C.byref(s), None, C.byref(h)), rbfl.E_INVALID_ARG, f"spec {label}")
        assert not h.value, label
    expect(lib.rbfl_build(None, None, None), rbfl.E_INVALID_ARG, "NULL spec")
    # several start-ups: argument checks, and a broken second spec fails the
    # call before any device work with every output left NULL
    lib.rbfl_build_many.argtypes = [C.POINTER(rbfl.BuildSpec), C.c_int32, C.c_int32, C.c_void_p,
                                    C.POINTER(C.c_void_p)]
    pair = (rbfl.BuildSpec * 2)(spec(), spec())
    pair[1].q = 0
    outs = (C.c_void_p * 2)()
    expect(lib.rbfl_build_many(pair, 2, 2, None, outs), rbfl.E_INVALID_ARG, "build_many broken second spec")
    assert not outs[0] and not outs[1]
    expect(lib.rbfl_build_many(None, 1, 1, None, outs), rbfl.E_INVALID_ARG, "build_many NULL specs")
    expect(lib.rbfl_build_many(pair, 0, 1, None, outs), rbfl.E_INVALID_ARG, "build_many n = 0")
    expect(lib.rbfl_build_many(pair, 1, 0, None, outs), rbfl.E_INVALID_ARG, "build_many no threads")
    expect(lib.rbfl_build_many(pair, 1, 1, None, None), rbfl.E_INVALID_ARG, "build_many NULL out")

    # ---- NULL handles and arguments
    nul = C.c_void_p()
    buf = (C.c_double * 8)()
    expect(lib.rbfl_eval(nul, buf, C.c_int64(1), buf, 0, nul), rbfl.E_INVALID_ARG, "eval NULL handle")
    expect(lib.rbfl_interp(nul, buf, C.c_int64(1), buf, 0, nul), rbfl.E_INVALID_ARG, "interp NULL handle")
    expect(lib.rbfl_brute(nul, buf, C.c_int64(1), buf, nul), rbfl.E_INVALID_ARG, "brute NULL handle")
    expect(lib.rbfl_query(nul, 0, buf, C.c_size_t(64)), rbfl.E_INVALID_ARG, "query NULL handle")
    expect(lib.rbfl_save(nul, b"/nonexistent"), rbfl.E_INVALID_ARG, "save NULL handle")
    expect(lib.rbfl_eval_static(nul, buf, C.c_int64(1), buf, nul), rbfl.E_INVALID_ARG, "static NULL handle")
    expect(lib.rbfl_fuse_epilogue(nul, 1), rbfl.E_INVALID_ARG, "fuse NULL handle")
    lib.rbfl_set_split_tol.argtypes = [C.c_void_p, C.c_double]
    expect(lib.rbfl_set_split_tol(nul, C.c_double(5e-4)), rbfl.E_INVALID_ARG, "split tol NULL handle")
    expect(lib.rbfl_eval_ragged(None, 1, None, None, None, nul), rbfl.E_INVALID_ARG, "ragged NULL")
    counts = (C.c_int64 * 1)(1)
    out = C.c_void_p()
    expect(lib.rbfl_plan_create(None, 1, counts, buf, buf, 0, nul, C.byref(out)), rbfl.E_INVALID_ARG,
           "plan NULL handles")
    expect(lib.rbfl_mlp_create(0, 8, 8, buf, C.byref(out)), rbfl.E_INVALID_ARG, "mlp sizes")
    expect(lib.rbfl_sampler_create(nul, None, None, nul, C.byref(out)), rbfl.E_INVALID_ARG, "sampler NULL")
    expect(lib.rbfl_destroy(nul), rbfl.OK, "destroy NULL")

    # ---- host-only queries
    for form, want in ((rbfl.FORM_SPLIT, 4),):
        n_checks += 1
        assert lib.rbfl_variants(form) == want
    assert lib.rbfl_variants(99) < 0

    # ---- store parsing: missing, damaged and fuzzed files
    import tempfile
    rng = np.random.default_rng(2024)
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "f.rbfl").encode()
        h = C.c_void_p()
        expect(lib.rbfl_load(os.path.join(d, "missing").encode(), None, C.byref(h)), rbfl.E_INVALID_ARG,
               "missing store")
        base = store_file([(t, 8, bytes(rng.integers(0, 256, 64, dtype=np.uint8))) for t in range(1, 16)])
        cases = [b"", b"RBFLSTOR", base[:-3], base + b"x", store_file([], fmt=2), store_file([], abi=0), base]
        for _ in range(300):
            b = bytearray(base)
            for _ in range(int(rng.integers(1, 6))):
                b[int(rng.integers(0, len(b)))] = int(rng.integers(0, 256))
            cases.append(bytes(b))
            # plausible section headers with huge or zero counts and sizes
            t = int(rng.integers(1, 16))
            es = [0, 1, 8, 16, 1 << 31][int(rng.integers(0, 5))]
            cnt = [0, 1, 1 << 40, (1 << 64) - 1][int(rng.integers(0, 4))]
            head = b"RBFLSTOR" + struct.pack("<IIQ", 1, rbfl.ABI_VERSION, int(rng.integers(1, 20)))
            cases.append(with_checksum(head + struct.pack("<IIQ", t, es, cnt) + bytes(int(rng.integers(0, 64)))))
        for i, data in enumerate(cases):
            with open(p, "wb") as f:
                f.write(data)
            expect(lib.rbfl_load(p, None, C.byref(h)), rbfl.E_INVALID_ARG, f"damaged store {i}")
            assert not h.value
    print(f"host checks: {n_checks} passed", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
