"""GPU: the no-allocation entry point sw_sweep_static (library-held scratch)
gives exactly what sw_init + sw_load_spins + sw_sweep + sw_measure give, on two
calls in a row, the second on a smaller lattice."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1208_2080_amd import binding
from paper_1208_2080_amd import workloads as wl

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def say(msg):
    print(msg, flush=True)


def _static_sweep(L, q, K, seed, spins, first, n, tile_rows=0, measure=True):
    params = binding.make_params(L, q, K, seed, True, 2, tile_rows)
    dev_spins = torch.from_numpy(np.ascontiguousarray(spins, dtype=np.uint8).reshape(-1)).to("cuda:0")
    dev_obs = torch.full((n, 2 + q), -7, dtype=torch.int64, device="cuda:0") if measure else None
    dev_status = torch.full((1,), 12345, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()
    stream.synchronize()
    rc = binding.lib().sw_sweep_static(ctypes.byref(params), ctypes.c_void_p(dev_spins.data_ptr()), first, n,
                                       ctypes.c_void_p(dev_obs.data_ptr()) if measure else None,
                                       ctypes.c_void_p(dev_status.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    binding._check(rc)
    out_spins = dev_spins.cpu().numpy().reshape(L, L)
    out_obs = dev_obs.cpu().numpy() if measure else None
    return out_spins, out_obs, int(dev_status.cpu().item())


def _plain_sweep(L, q, K, seed, spins, first, n, tile_rows=0):
    lat = binding.Lattice(L, q, K, seed=seed, obs_capacity=max(2, n), tile_rows=tile_rows)
    lat.load_spins(spins, first)
    lat.sweep(n)
    out = lat.spins(), lat.measure(first, n)
    lat.close()
    return out


@pytest.mark.parametrize("tile_rows", [0, 32, 128])
def test_static_matches_workspace_path_twice(tile_rows):
    cases = [(300, 3, wl.critical_coupling(3), 5, 7, 6), (100, 2, wl.critical_coupling(2), 9, 0, 4)]
    for L, q, K, seed, first, n in cases:
        say(f"static L={L} q={q} seed={seed} first={first} n={n} ty={tile_rows}")
        rng = np.random.Generator(np.random.PCG64(L + seed))
        start = rng.integers(0, q, (L, L), dtype=np.uint8)
        s_ref, obs_ref = _plain_sweep(L, q, K, seed, start, first, n, tile_rows)
        s_got, obs_got, status = _static_sweep(L, q, K, seed, start, first, n, tile_rows)
        assert status == 0
        assert np.array_equal(s_got, s_ref), f"spins differ (L={L})"
        assert np.array_equal(obs_got, obs_ref), f"observables differ (L={L})"


def test_static_without_measurement_and_limits():
    L, q, K, seed = 130, 4, wl.critical_coupling(4), 3
    start = np.random.Generator(np.random.PCG64(1)).integers(0, q, (L, L), dtype=np.uint8)
    s_ref, _ = _plain_sweep(L, q, K, seed, start, 2, 3)
    s_got, _, status = _static_sweep(L, q, K, seed, start, 2, 3, measure=False)
    assert status == 0 and np.array_equal(s_got, s_ref)
    # beyond the scratch: a clear error, nothing launched
    params = binding.make_params(4096, 2, K, seed)
    rc = binding.lib().sw_sweep_static(ctypes.byref(params), ctypes.c_void_p(1), 0, 1, None, None, None)
    assert rc == binding.SW_ESPACE and b"scratch" in binding.lib().sw_last_error()
