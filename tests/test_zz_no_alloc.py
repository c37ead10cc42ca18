"""sw_sweep_noalloc (the sweep that allocates nothing) against sw_sweep of a
sim in the same state: spins and record equal bit for bit, on calls in a row
whose lattices shrink (the static scratch keeps the previous call's
contents), on a chain of calls that feeds each output back in, and at the
largest lattice the scratch holds."""
import math

import numpy as np
import pytest

import paper_2302_14720_amd as sw

pytestmark = pytest.mark.gpu

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0


def _state(L, beta, seed, sweeps):
    """Spins of a hot-started sim after `sweeps` sweeps (a realistic input)."""
    with sw.Sim(L, beta, 1.0, seed) as s:
        s.sweep(sweeps)
        return s.spins()


def _reference(L, beta, seed, t, spins, n=1):
    with sw.Sim(L, beta, 1.0, seed) as s:
        s.set_spins(spins, t)
        s.sweep(n)
        return s.spins(), s.series(t, n)


def _noalloc(L, beta, seed, t, dev_spins, torch, stream):
    rec = torch.zeros(sw.OBS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    print(f"[noalloc] L={L} beta={beta:.6f} seed={seed} t={t}", flush=True)
    sw.sw_sweep_noalloc(L, beta, 1.0, seed, t, dev_spins.data_ptr(), rec.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    return dev_spins.cpu().numpy().copy(), np.frombuffer(rec.cpu().numpy().tobytes(), dtype=sw.OBS_DTYPE)[0]


@pytest.fixture(scope="module")
def torch_stream():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch, torch.cuda.Stream()


def test_two_calls_second_smaller(torch_stream):
    torch, stream = torch_stream
    for L, beta, seed, t in ((512, BETA_C, 21, 6), (128, 0.3, 22, 3)):
        spins = _state(L, beta, seed, t)
        want_spins, want_rec = _reference(L, beta, seed, t, spins)
        dev = torch.from_numpy(spins).to("cuda")
        got_spins, got_rec = _noalloc(L, beta, seed, t, dev, torch, stream)
        assert np.array_equal(got_spins, want_spins), f"L={L}: spins differ"
        assert got_rec.tobytes() == want_rec[0].tobytes(), f"L={L}: records differ"


def test_chain_matches_consecutive_sweeps(torch_stream):
    torch, stream = torch_stream
    L, seed, t0, n = 256, 31, 2, 5
    spins = _state(L, BETA_C, seed, t0)
    want_spins, want_recs = _reference(L, BETA_C, seed, t0, spins, n)
    dev = torch.from_numpy(spins).to("cuda")
    for k in range(n):
        got_spins, got_rec = _noalloc(L, BETA_C, seed, t0 + k, dev, torch, stream)
        assert got_rec.tobytes() == want_recs[k].tobytes(), f"record of sweep {t0 + k} differs"
    assert np.array_equal(got_spins, want_spins)


def test_largest_lattice_then_smallest(torch_stream):
    torch, stream = torch_stream
    for L, beta, seed, t in ((2048, BETA_C, 41, 1), (32, 0.6, 42, 9)):
        spins = _state(L, beta, seed, t)
        want_spins, want_rec = _reference(L, beta, seed, t, spins)
        dev = torch.from_numpy(spins).to("cuda")
        got_spins, got_rec = _noalloc(L, beta, seed, t, dev, torch, stream)
        assert np.array_equal(got_spins, want_spins), f"L={L}: spins differ"
        assert got_rec.tobytes() == want_rec[0].tobytes(), f"L={L}: records differ"


def test_rejects_what_the_scratch_cannot_hold(torch_stream):
    torch, stream = torch_stream
    dev = torch.ones(4096 * 4096, dtype=torch.int8, device="cuda")
    rec = torch.zeros(sw.OBS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    with pytest.raises(sw.SwError) as e:
        sw.sw_sweep_noalloc(4096, BETA_C, 1.0, 1, 0, dev.data_ptr(), rec.data_ptr(), stream.cuda_stream)
    assert e.value.code == sw.SW_ERANGE
    with pytest.raises(sw.SwError) as e:
        sw.sw_sweep_noalloc(48, BETA_C, 1.0, 1, 0, dev.data_ptr(), rec.data_ptr(), stream.cuda_stream)
    assert e.value.code == sw.SW_EINVAL
    with pytest.raises(sw.SwError) as e:
        sw.sw_sweep_noalloc(64, BETA_C, 1.0, 1, 0, 0, rec.data_ptr(), stream.cuda_stream)
    assert e.value.code == sw.SW_EINVAL
    with pytest.raises(sw.SwError) as e:
        sw.sw_sweep_noalloc(64, BETA_C, 1.0, 1, 0, dev.data_ptr() + 1, rec.data_ptr(), stream.cuda_stream)
    assert e.value.code == sw.SW_EINVAL
