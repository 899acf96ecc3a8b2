"""Rounding of the 2-byte storage types, through the C ABI.

lbm_set_populations stores f^n so that the next pull returns it; on a fully
periodic lattice every population maps to one stored element, so a round trip
through lbm_set_populations and lbm_get_populations returns exactly the
stored value.  Each FP64 value is taken to FP32 (round to nearest even), then
to the storage type: FP16 by the hardware conversion, BF16 by round to
nearest even on the top 16 bits (ties to the even kept bit, NaN excluded).
The expected bits are computed here on the host with integer arithmetic;
the inputs cover random FP32 patterns over the whole finite range, exact
ties with an even and an odd kept bit, values one unit either side of a tie,
denormals and the largest finite values (which round to infinity in BF16
when they pass the largest BF16 number by half a unit or more).
"""
import numpy as np
import pytest

from gpu_common import banner
from paper_2511_01629_amd import lbm

pytestmark = pytest.mark.gpu

NX, NY, Q = 64, 48, 9


def _patterns(rng, n):
    """n finite FP32 bit patterns (uint32)."""
    r = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    exp = (r >> 23) & 0xFF
    r = np.where(exp == 0xFF, r & ~np.uint32(0x40000000), r)  # no Inf/NaN: clear an exponent bit
    hi = rng.integers(0, 2 ** 16, size=n, dtype=np.uint64).astype(np.uint32)
    hi = np.where(((hi >> 7) & 0xFF) == 0xFF, hi & np.uint32(0xBFFF), hi)  # finite high halves
    k = n // 8
    r[0:k] = (hi[0:k] << 16) | 0x8000                    # exact ties (even and odd kept bits)
    r[k:2 * k] = (hi[k:2 * k] << 16) | 0x7FFF            # one unit below a tie
    r[2 * k:3 * k] = (hi[2 * k:3 * k] << 16) | 0x8001    # one unit above a tie
    r[3 * k:4 * k] = r[3 * k:4 * k] & np.uint32(0x807FFFFF)  # denormals and zeros
    r[4 * k:4 * k + 4] = np.array([0x7F7FFFFF, 0xFF7FFFFF, 0x7F7F8000, 0x7F7F7FFF], dtype=np.uint32)
    return r


def _bf16_rne(bits):
    b = bits.astype(np.uint64)
    return (((b + 0x7FFF + ((b >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint32)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_two_byte_storage_rounds_to_nearest_even(storage):
    banner(f"storage rounding {storage}")
    rng = np.random.default_rng(2511 if storage == "bf16" else 2512)
    bits = _patterns(rng, NX * NY * Q)
    x32 = bits.view(np.float32)
    if storage == "f16":
        # FP16 covers a narrower range: keep the values it represents without overflow
        x32 = np.clip(x32, np.float32(-65504.0), np.float32(65504.0))
        x32 = np.where(np.isfinite(x32), x32, np.float32(0.0)).astype(np.float32)
    f = x32.astype(np.float64).reshape(1, NY, NX, Q)
    cfg = dict(lattice="D2Q9", n=(NX, NY, 1), periodic=(1, 1, 0), tau=0.8)
    sim = lbm.Simulation(cfg, [], storage=storage)
    sim.set_populations(f)
    g = sim.populations()
    sim.close()
    if storage == "bf16":
        want = (_bf16_rne(x32.reshape(-1).view(np.uint32)) << 16).view(np.float32).astype(np.float64)
    else:
        want = x32.reshape(-1).astype(np.float16).astype(np.float64)  # numpy: round to nearest even
    got = g.reshape(-1)
    same = (got == want) | (np.isnan(got) & np.isnan(want))
    assert same.all(), (np.flatnonzero(~same)[:5], got[~same][:5], want[~same][:5])
    # the ties really were ties, and some rounded up, some down
    if storage == "bf16":
        k = f.size // 8
        t = x32.reshape(-1)[:k].view(np.uint32)
        up = (_bf16_rne(t) << 16) > (t & np.uint32(0xFFFF0000))
        assert 0 < up.sum() < k
