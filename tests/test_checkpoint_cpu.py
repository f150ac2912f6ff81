"""mps_restore validates a checkpoint image on the host before any device
call.  The images here are written by this file from the format that
include/ptebd.h and the library describe (64-byte header, chi, Schmidt
values, site tensors, 64-bit FNV-1a checksum), not by the library, so a
valid one pins that format: it passes every check and only then fails, for
want of a GPU, at device set-up."""
import ctypes
import struct

import numpy as np
import pytest

FNV_BASIS = 14695981039346656037
FNV_PRIME = 1099511628211
MASK = (1 << 64) - 1


def fnv_words(data: bytes, h: int = FNV_BASIS) -> int:
    """FNV-1a over little-endian 8-byte words, the tail bytes one at a time."""
    n8 = len(data) // 8 * 8
    for (w,) in struct.iter_unpack("<Q", data[:n8]):
        h = ((h ^ w) * FNV_PRIME) & MASK
    for b in data[n8:]:
        h = ((h ^ b) * FNV_PRIME) & MASK
    return h


def image(L, d, chi, phys_L=None, phys_d=None, supersite=0, u1=0, ledger=0.0, version=1, tag=b"ptebdck\0",
          seed=0, payload_delta=0, fix_checksum=True):
    phys_L = L if phys_L is None else phys_L
    phys_d = d if phys_d is None else phys_d
    rng = np.random.default_rng(seed)
    chi_b = np.asarray(chi, dtype="<i4").tobytes()
    chi_b += b"\0" * (-len(chi_b) % 8)
    lam = np.concatenate([np.sort(rng.random(c))[::-1] for c in chi]).astype("<f8").tobytes()
    B = b"".join(rng.standard_normal(2 * chi[i] * d * chi[i + 1]).astype("<f8").tobytes() for i in range(L))
    body = chi_b + lam + B
    hdr = lambda ck: (tag + struct.pack("<I", version) + struct.pack("<7i", L, d, phys_L, phys_d, supersite, u1, 0)
                      + struct.pack("<d", ledger) + struct.pack("<QQ", len(body) + payload_delta, ck))
    assert len(hdr(0)) == 64
    ck = fnv_words(body[:len(body) + min(payload_delta, 0)], fnv_words(hdr(0))) if fix_checksum else 12345
    return hdr(ck) + body


@pytest.fixture(scope="module")
def pt():
    import paper_2401_05301_amd as pt
    return pt


def restore_status(pt, img, L=6, d=3, chi_max=8, supersite=False, u1=False):
    model = pt.make_model(L, d, 1.0)
    opts = pt.make_opts(chi_max=chi_max, supersite=supersite, u1=u1)
    with pytest.raises(pt.TebdError) as e:
        pt.mps_restore(model, opts, img)
    return e.value.status, str(e.value)


CHI6 = [1, 3, 8, 8, 8, 3, 1]


def test_valid_image_passes_host_checks(pt):
    """A well-formed image passes every host check: without a GPU only device
    set-up stops it (TEBD_EDEVICE); with one it loads."""
    for img, kw in ((image(6, 3, CHI6, ledger=1e-9), {}),
                    (image(3, 9, [1, 8, 8, 1], phys_L=6, phys_d=3, supersite=1), dict(supersite=True))):
        opts = pt.make_opts(chi_max=8, **kw)
        try:
            h = pt.mps_restore(pt.make_model(6, 3, 1.0), opts, img)
        except pt.TebdError as e:
            assert e.status == pt.TEBD_EDEVICE, str(e)
        else:
            pt.mps_free(h)


@pytest.mark.parametrize("kw, opt, words", [
    (dict(tag=b"ptebdcX\0"), {}, "not a checkpoint"),
    (dict(version=2), {}, "version"),
    (dict(supersite=1), {}, "supersite"),
    (dict(phys_L=8), {}, "L or d"),
    (dict(phys_d=4), {}, "L or d"),
    (dict(payload_delta=8), {}, "cut short"),
    (dict(payload_delta=-8), {}, "size does not match"),
    (dict(fix_checksum=False), {}, "checksum"),
    (dict(ledger=-1.0), {}, "ledger"),
    ({}, dict(chi_max=4), "bond dimension"),
])
def test_bad_images_are_refused(pt, kw, opt, words):
    st, msg = restore_status(pt, image(6, 3, CHI6, **kw), **opt)
    assert st == pt.TEBD_EINVAL and words in msg, msg


def test_damaged_and_cut_images_are_refused(pt):
    good = bytearray(image(6, 3, CHI6))
    for pos in (44, 70, len(good) // 2, len(good) - 1):
        bad = bytearray(good)
        bad[pos] ^= 0x10
        st, msg = restore_status(pt, bytes(bad))
        assert st == pt.TEBD_EINVAL and "checksum" in msg, (pos, msg)
    for n in (0, 63, 64, len(good) - 1):
        st, msg = restore_status(pt, bytes(good[:n]))
        assert st == pt.TEBD_EINVAL and "cut short" in msg, (n, msg)


def test_bond_edges_must_be_one(pt):
    st, msg = restore_status(pt, image(6, 3, [3, 3, 8, 8, 8, 3, 1]))
    assert st == pt.TEBD_EINVAL and "chi[0]" in msg


def test_null_arguments(pt):
    lib = pt._lib
    model, opts = pt.make_model(6, 3, 1.0), pt.make_opts(chi_max=8)
    h = ctypes.c_void_p()
    assert lib.mps_restore(ctypes.byref(model), ctypes.byref(opts), None, 0, ctypes.byref(h)) == pt.TEBD_EINVAL
    n = ctypes.c_size_t()
    assert lib.mps_checkpoint(None, None, 0, ctypes.byref(n)) == pt.TEBD_EINVAL
