"""Host-only tests of the files the runtime keeps between processes: the tile-cache file (save,
load, merge, key mismatch, damage) and the cost-model file's checks (a file written here from
the documented layout, then truncated, altered, or holding non-finite values)."""
import os
import struct

import numpy as np
import pytest

import paper_2009_07482_amd as psc

F, H, P = psc.PSC_FEATURES, 64, psc.PSC_MLP_PARAMS


def fnv1a64(b):
    h = 0xcbf29ce484222325
    for x in b:
        h ^= x
        h = (h * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def mlp_file(step=3, params=None, m=None, v=None, mean=None, std=None):
    g = np.random.default_rng(0)
    params = g.standard_normal(P).astype(np.float32) if params is None else params
    m = g.standard_normal(P).astype(np.float32) if m is None else m
    v = np.abs(g.standard_normal(P)).astype(np.float32) if v is None else v
    mean = np.zeros(F, np.float32) if mean is None else mean
    std = np.ones(F, np.float32) if std is None else std
    body = b"PSCMLP01" + struct.pack("<IIIIq", F, H, P, 0, step)
    for a in (mean, std, params, m, v):
        body += np.asarray(a, "<f4").tobytes()
    return body + struct.pack("<Q", fnv1a64(body))


@pytest.fixture
def tmp(tmp_path):
    return str(tmp_path)


def _write(path, b):
    with open(path, "wb") as fh:
        fh.write(b)
    return path


def test_mlp_file_accepted(tmp):
    assert psc.psc_mlp_file_check(_write(os.path.join(tmp, "ok.bin"), mlp_file(step=7))) == 7


@pytest.mark.parametrize("damage", ["truncated", "bitflip", "magic", "shape", "nan_param", "inf_moment",
                                    "neg_second_moment", "zero_std", "neg_step", "missing"])
def test_mlp_file_refused(tmp, damage):
    b = bytearray(mlp_file())
    path = os.path.join(tmp, "bad.bin")
    if damage == "truncated":
        b = b[:-100]
    elif damage == "bitflip":
        b[2000] ^= 0x10
    elif damage == "magic":
        b[0:8] = b"PSCMLP02"
        b = b[:-8] + struct.pack("<Q", fnv1a64(bytes(b[:-8])))
    elif damage == "shape":
        b = bytearray(b"PSCMLP01" + struct.pack("<IIIIq", F, 32, P, 0, 3)) + b[32:]
        b = b[:-8] + struct.pack("<Q", fnv1a64(bytes(b[:-8])))
    elif damage in ("nan_param", "inf_moment", "neg_second_moment", "zero_std", "neg_step"):
        # well-formed, checksum correct, values unusable
        p = np.zeros(P, np.float32)
        m = np.zeros(P, np.float32)
        v = np.zeros(P, np.float32)
        std = np.ones(F, np.float32)
        step = 3
        if damage == "nan_param":
            p[17] = np.nan
        elif damage == "inf_moment":
            m[5] = np.inf
        elif damage == "neg_second_moment":
            v[9] = -1.0
        elif damage == "zero_std":
            std[4] = 0.0
        else:
            step = -1
        b = mlp_file(step=step, params=p, m=m, v=v, std=std)
    if damage != "missing":
        _write(path, bytes(b))
    with pytest.raises(psc.PscError) as e:
        psc.psc_mlp_file_check(path)
    assert e.value.status == psc.PSC_ERR_IO


def test_tile_cache_roundtrip_and_merge(tmp):
    path = os.path.join(tmp, "tiles.txt")
    psc.psc_tile_cache_clear()
    psc.psc_tile_cache_set(1024, 64, 1024, "bf16", "bf16", 14)
    psc.psc_tile_cache_set(512, 512, 64, "f32", "f32", 3)
    psc.psc_tile_cache_save(path, "archA/hip1")
    assert psc.psc_tile_cache_clear() == 2
    psc.psc_tile_cache_set(512, 512, 64, "f32", "f32", 5)     # replaced by the file's choice
    psc.psc_tile_cache_set(7, 7, 7, "f32", "f32", 2)          # kept
    assert psc.psc_tile_cache_load(path, "archA/hip1") == 2
    assert psc.psc_tile_cache_get(1024, 64, 1024, "bf16", "bf16") == 14
    assert psc.psc_tile_cache_get(512, 512, 64, "f32", "f32") == 3
    assert psc.psc_tile_cache_get(7, 7, 7, "f32", "f32") == 2
    psc.psc_tile_cache_clear()


def test_tile_cache_other_key_loads_nothing(tmp):
    path = os.path.join(tmp, "tiles.txt")
    psc.psc_tile_cache_clear()
    psc.psc_tile_cache_set(256, 256, 256, "f32", "f32", 2)
    psc.psc_tile_cache_save(path, "gfx950/hip70200000")
    psc.psc_tile_cache_clear()
    with pytest.raises(psc.PscError) as e:
        psc.psc_tile_cache_load(path, "gfx942/hip70200000")
    assert e.value.status == psc.PSC_ERR_STATE
    assert psc.psc_tile_cache_get(256, 256, 256, "f32", "f32") == 0


@pytest.mark.parametrize("damage", ["edited_entry", "bad_tile", "no_checksum", "garbage", "missing"])
def test_tile_cache_damage_loads_nothing(tmp, damage):
    path = os.path.join(tmp, "tiles.txt")
    psc.psc_tile_cache_clear()
    psc.psc_tile_cache_set(128, 128, 128, "f32", "f32", 4)
    psc.psc_tile_cache_set(64, 64, 64, "bf16", "f32", 2)
    psc.psc_tile_cache_save(path, "k")
    psc.psc_tile_cache_clear()
    text = open(path).read()
    if damage == "edited_entry":
        text = text.replace("entry 128 128 128 0 0 4", "entry 128 128 128 0 0 5")
    elif damage == "bad_tile":
        body = text[: text.rindex("checksum ")].replace("entry 128 128 128 0 0 4", "entry 128 128 128 0 0 99")
        text = body + "checksum %016x\n" % fnv1a64(body.encode())
    elif damage == "no_checksum":
        text = text[: text.rindex("checksum ")]
    elif damage == "garbage":
        text = "hello\n"
    if damage == "missing":
        os.remove(path)
    else:
        open(path, "w").write(text)
    with pytest.raises(psc.PscError) as e:
        psc.psc_tile_cache_load(path, "k")
    assert e.value.status == psc.PSC_ERR_IO
    assert psc.psc_tile_cache_get(128, 128, 128, "f32", "f32") == 0
    assert psc.psc_tile_cache_get(64, 64, 64, "bf16", "f32") == 0


def test_tile_cache_key_must_be_a_word(tmp):
    with pytest.raises(psc.PscError) as e:
        psc.psc_tile_cache_save(os.path.join(tmp, "t.txt"), "two words")
    assert e.value.status == psc.PSC_ERR_ARG
