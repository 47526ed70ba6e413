"""The C ABI library: symbols and host-side argument checks (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1911_04200_amd import jas

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "jas.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jas_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = jas.load()
    names = declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), f"{name} missing from libjas.so"
    assert sorted(jas.EXPORTS) == names


def test_flag_and_status_values_match_the_header():
    text = open(os.path.join(ROOT, "include", "jas.h")).read()
    flags = dict(re.findall(r"#define (JAS_\w+) (0x[0-9a-fA-F]+)u", text))
    assert len(flags) >= 6
    for name, value in flags.items():
        assert getattr(jas, name) == int(value, 16), name
    for name, value in re.findall(r"(JAS_E\w+|JAS_OK)\s*=\s*(-?\d+)", text):
        assert getattr(jas, name) == int(value), name


def test_struct_fields_match_the_header():
    """The binding's structs list the header's fields, in order and with their widths."""
    text = open(os.path.join(ROOT, "include", "jas.h")).read()
    for cname, cls in (("jas_encode_opts", jas.jas_encode_opts), ("jas_encode_stats", jas.jas_encode_stats)):
        body = re.search(r"typedef struct \{((?:(?!typedef struct).)*?)\} " + cname + ";", text, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"uint(32|64)_t (\w+);", body)
        assert [(n, int(w)) for w, n in fields] == [(n, ctypes.sizeof(t) * 8) for n, t in cls._fields_], cname


def test_gram_variant_flag_matches_the_header():
    text = open(os.path.join(ROOT, "include", "jas.h")).read()
    assert "#define JAS_GRAM_VARIANT(v) ((((uint32_t)(v)) + 1u) << 16)" in text
    assert jas.JAS_GRAM_VARIANT(0) == 1 << 16 and jas.JAS_GRAM_VARIANT(9) == 10 << 16
    assert jas.jas_gram_variants() >= 2


def test_version():
    assert "gfx950" in jas.jas_version()


def _opts(U=24, flags=jas.JAS_HOST_PTRS, **kw):
    return jas.jas_encode_opts(U, kw.get("batch_bits", 0), kw.get("dmin", 0), flags, kw.get("budget", 0))


@pytest.mark.parametrize("offsets,msg", [([1, 3], "offsets[0]"), ([0, 3, 2], "decrease")])
def test_encode_rejects_bad_host_offsets(offsets, msg):
    ids = np.arange(3, dtype=np.uint64)
    with pytest.raises(jas.JasError) as e:
        jas.jas_encode(ids, np.array(offsets, dtype=np.uint64), len(offsets) - 1, _opts())
    assert e.value.status == jas.JAS_EINVAL and msg in e.value.message


@pytest.mark.parametrize("U", [0, 64, 100])
def test_encode_rejects_universe_bits(U):
    ids = np.arange(3, dtype=np.uint64)
    with pytest.raises(jas.JasError) as e:
        jas.jas_encode(ids, np.array([0, 3], dtype=np.uint64), 1, _opts(U=U))
    assert e.value.status == jas.JAS_EINVAL


def test_encode_rejects_key_overflow():
    # 2^20 sets need 20 sample bits: U = 50 leaves no room in a 64-bit key
    n = 1 << 20
    off = np.zeros(n + 1, dtype=np.uint64)
    with pytest.raises(jas.JasError) as e:
        jas.jas_encode(np.zeros(1, np.uint64), off, n, _opts(U=50))
    assert e.value.status == jas.JAS_EINVAL and "exceeds 64" in e.value.message


def test_null_arguments():
    lib = jas.load()
    st = jas.jas_encode_stats()
    assert lib.jas_encode(None, None, 1, None, None, None, ctypes.byref(st)) == jas.JAS_EINVAL
    out = ctypes.c_void_p()
    assert lib.jas_encode(None, None, 1, None, None, ctypes.byref(out), None) == jas.JAS_EINVAL
    assert "opts" in jas.jas_last_error()
    o = _opts()
    assert lib.jas_encode(None, None, -1, ctypes.byref(o), None, ctypes.byref(out), None) == jas.JAS_EINVAL
    assert lib.jas_encode(None, None, 2, ctypes.byref(o), None, ctypes.byref(out), None) == jas.JAS_EINVAL
    assert lib.jas_gram(None, 0, None, None, None, None, None) == jas.JAS_EINVAL
    assert lib.jas_query(None, None, None, 1, 0, None, None, None, None, None) == jas.JAS_EINVAL
    assert lib.jas_db_size(None) == -1
    assert lib.jas_db_stats(None, ctypes.byref(st)) == jas.JAS_EINVAL
    assert lib.jas_query_workspace_bytes(None, 1, 10) == 0
    lib.jas_db_free(None)


def test_error_message_is_thread_local_and_reset():
    lib = jas.load()
    assert lib.jas_gram(None, 0, None, None, None, None, None) == jas.JAS_EINVAL
    assert jas.jas_last_error() != ""
    st = jas.jas_encode_stats()
    # a call that fails differently replaces the message
    assert lib.jas_db_stats(None, ctypes.byref(st)) == jas.JAS_EINVAL
    assert "jas_db_stats" in jas.jas_last_error()


def test_finalize_argument_checks():
    lib = jas.load()
    assert lib.jas_finalize(-1, 0, None, None, None, None, None) == jas.JAS_EINVAL
    assert lib.jas_finalize(4, jas.JAS_TUNE, None, None, None, None, None) == jas.JAS_EINVAL
    assert "JAS_UPPER" in jas.jas_last_error()
    assert lib.jas_finalize(4, 0, None, None, None, None, None) == jas.JAS_EINVAL
    assert lib.jas_finalize(0, 0, None, None, None, None, None) == jas.JAS_OK


def test_card_limit_and_its_test_hook(monkeypatch):
    """2^31 by default; JAS_TEST_CARD_LIMIT lowers it, and values that are not
    a positive integer below 2^31 are ignored."""
    monkeypatch.delenv("JAS_TEST_CARD_LIMIT", raising=False)
    assert jas.jas_card_limit() == 1 << 31
    for value, want in [("100", 100), ("1", 1), (str((1 << 31) - 1), (1 << 31) - 1), (str(1 << 31), 1 << 31),
                        ("0", 1 << 31), ("-5", 1 << 31), ("12x", 1 << 31), ("", 1 << 31)]:
        monkeypatch.setenv("JAS_TEST_CARD_LIMIT", value)
        assert jas.jas_card_limit() == want, value


def test_db_part_constants_and_null_db():
    text = open(os.path.join(ROOT, "include", "jas.h")).read()
    parts = dict(re.findall(r"#define (JAS_DB_\w+) (\d+)\n", text))
    assert len(parts) == 6
    for name, value in parts.items():
        assert getattr(jas, name) == int(value), name
    lib = jas.load()
    assert lib.jas_db_part_size(None, jas.JAS_DB_WORDS) == 0
    assert lib.jas_db_read(None, jas.JAS_DB_WORDS, 0, 0, None) == jas.JAS_EINVAL


def test_encode_rejects_a_bad_word_width():
    ids = np.arange(3, dtype=np.uint64)
    for wb in (16, 48, 128):
        opts = jas.jas_encode_opts(24, 0, 0, jas.JAS_HOST_PTRS, 0, wb)
        with pytest.raises(jas.JasError) as e:
            jas.jas_encode(ids, np.array([0, 3], dtype=np.uint64), 1, opts)
        assert e.value.status == jas.JAS_EINVAL and "word_bits" in e.value.message


def test_query_only_needs_the_query_index():
    ids = np.arange(3, dtype=np.uint64)
    opts = jas.jas_encode_opts(24, 0, 0, jas.JAS_HOST_PTRS | jas.JAS_QUERY_ONLY, 0)
    with pytest.raises(jas.JasError) as e:
        jas.jas_encode(ids, np.array([0, 3], dtype=np.uint64), 1, opts)
    assert e.value.status == jas.JAS_EINVAL and "JAS_KEEP_IDS" in e.value.message
