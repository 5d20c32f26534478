"""The schedule cache (host code of libqft.so, driven here through the CPU
emulation library that compiles the same header): store and lookup, the
versioned format, and that a missing, corrupted or foreign file is ignored
rather than trusted."""
import ctypes
import json
import os

import pytest

from tests.emu import build as EB


@pytest.fixture(scope="module")
def emu():
    return EB.load()


def _lookup(emu, path, key):
    buf = ctypes.create_string_buffer(256)
    found = emu.emu_cache_lookup(path.encode(), key.encode(), buf, 256)
    return buf.value.decode() if found else None


def test_store_and_lookup(emu, tmp_path):
    path = str(tmp_path / "sub" / "dir" / "schedules.json")  # directories are created
    assert _lookup(emu, path, "k1") is None
    assert emu.emu_cache_store(path.encode(), b"gfx950/256cu/u/c32/16x256", b"two-pass/all")
    assert emu.emu_cache_store(path.encode(), b"gfx950/256cu/v/c32/4096:abc", b"t13:6-13+t14:14")
    assert _lookup(emu, path, "gfx950/256cu/u/c32/16x256") == "two-pass/all"
    assert _lookup(emu, path, "gfx950/256cu/v/c32/4096:abc") == "t13:6-13+t14:14"
    # overwrite keeps the other entry
    assert emu.emu_cache_store(path.encode(), b"gfx950/256cu/u/c32/16x256", b"two-pass")
    assert _lookup(emu, path, "gfx950/256cu/u/c32/16x256") == "two-pass"
    assert _lookup(emu, path, "gfx950/256cu/v/c32/4096:abc") == "t13:6-13+t14:14"
    # the file is plain JSON of the documented shape
    doc = json.load(open(path))
    assert doc["qft_schedule_cache"] == 1 and len(doc["entries"]) == 2


def test_corrupt_or_foreign_files_are_ignored(emu, tmp_path):
    path = str(tmp_path / "schedules.json")
    for text in ["", "not json", '{"qft_schedule_cache": 2, "entries": {"k": "v"}}',
                 '{"other": 1}', '{"qft_schedule_cache": 1, "entries": {"k": ']:
        with open(path, "w") as f:
            f.write(text)
        assert _lookup(emu, path, "k") is None, text
        # a store replaces what it cannot read
        assert emu.emu_cache_store(path.encode(), b"k", b"v")
        assert _lookup(emu, path, "k") == "v"


def test_rejects_names_that_would_break_the_format(emu, tmp_path):
    path = str(tmp_path / "schedules.json")
    assert not emu.emu_cache_store(path.encode(), b'bad"key', b"v")
    assert not emu.emu_cache_store(path.encode(), b"k", b"bad\\name")
    assert not os.path.exists(path)


def test_path_from_environment(emu, monkeypatch, tmp_path):
    buf = ctypes.create_string_buffer(4096)
    monkeypatch.setenv("QFT_SCHEDULE_CACHE", str(tmp_path / "x.json"))
    emu.emu_cache_path(buf, 4096)
    assert buf.value.decode() == str(tmp_path / "x.json")
    monkeypatch.setenv("QFT_SCHEDULE_CACHE", "off")
    assert emu.emu_cache_path(buf, 4096) == 0
    assert not emu.emu_cache_store(b"", b"k", b"v")   # disabled: nothing is written
    monkeypatch.delenv("QFT_SCHEDULE_CACHE")
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path / "xdg"))
    emu.emu_cache_path(buf, 4096)
    assert buf.value.decode() == str(tmp_path / "xdg" / "qft-gfx950" / "schedules.json")
