"""rfvr_mf_forward_static, the filter forward that allocates nothing, against
rfvr_mf_forward (same kernels, so the same bits) on two calls in a row, the
second smaller than the first (the static scratch keeps the first call's
contents), and its refusal of a call that needs more scratch than it has."""
import numpy as np
import pytest
import torch

from synth import freq_grid, line_points, planar_aperture

pytestmark = pytest.mark.gpu


def _inputs(dev, nx, ny, n_freq, lines, n_z, seed, jitter=None):
    from paper_2605_29097_amd import rfvr as R
    rng = np.random.default_rng(seed)
    f0, df = freq_grid(n_freq)
    tx = planar_aperture(nx, ny, 2e-3)
    if jitter:
        tx = tx + rng.uniform(-jitter, jitter, tx.shape).astype(np.float32)
    xyz, _ = line_points((0.0, 0.0, 0.30), 0.20, lines[0], lines[1], n_z, jitter_seed=seed)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    sig = [t(rng.normal(size=(nx * ny, n_freq, 2))) for _ in range(2)]
    return R.Aperture(tx=t(tx), f0=f0, df=df, n_freq=n_freq), t(xyz).view(-1, 3), sig


def test_static_filter_matches_workspace_filter(dev):
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    cases = [("1024 measurements x 128 frequencies, 2^20 points, two signals",
              _inputs(dev, 32, 32, 128, (64, 64), 256, 0), True),
             ("35 measurements x 45 frequencies, 4550 points, one signal",
              _inputs(dev, 7, 5, 45, (13, 5), 70, 1, jitter=2e-4), False)]
    for flags in (0, R.TERMS_DIRECT):
        for name, (ap, xq, sig), two in cases:
            print(f"[case] rfvr_mf_forward_static vs rfvr_mf_forward: {name}, flags {flags}", flush=True)
            s2 = sig[1] if two else None
            ref = R.mf_forward(ap, xq, sig[0], s2, flags=flags)
            nq = xq.shape[0]
            out = [torch.full((nq, 2), float("nan"), device=dev), torch.full((nq,), float("nan"), device=dev)]
            if two:
                out += [torch.full((nq, 2), float("nan"), device=dev), torch.full((nq,), float("nan"), device=dev)]
            got = R.mf_forward_static(ap, xq, sig[0], s2, flags=flags, out=out)
            torch.cuda.synchronize()
            assert len(got) == len(ref)
            for g, r in zip(got, ref):
                assert torch.equal(g, r), (name, flags, (g - r).abs().max().item())


def test_static_filter_refuses_oversized_call(dev):
    from paper_2605_29097_amd import rfvr as R
    R.lib()
    print("[case] rfvr_mf_forward_static refuses a call above its scratch", flush=True)
    ap, xq, sig = _inputs(dev, 128, 128, 256, (4, 4), 4, 2)
    assert R.lib().rfvr_mf_forward_ws_bytes(R.ctypes.byref(ap.c()), xq.shape[0], 1) > R.MF_STATIC_SCRATCH_BYTES
    z = torch.zeros(xq.shape[0], 2, device=dev)
    with pytest.raises(R.RfvrError, match="RFVR_E_INVALID"):
        R.mf_forward_static(ap, xq, sig[0], sig[1], out=[z, z[:, 0].contiguous(), z.clone(), z[:, 0].contiguous()])
