"""Chunk streaming of the two-temperature emission workload: line chunks
uploaded from host memory on a copy stream (double-buffered pinned staging)
while the previous chunk runs, sigma accumulated over the chunks.  The
streamed result equals the result of the same chunks resident on the device
(bitwise: same kernels, same order), and matches the oracle on the whole line
list at sampled points and around the strongest lines, for all four
(T_vib, T_rot) pairs, on the full 600,001-point grid."""
import numpy as np
import pytest

import oracle
import synth
from xs_helpers import X, log, make_plan, rel_err

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_streamed_chunks_equal_resident_and_oracle(prec):
    import torch
    P = X()
    wl = synth.workload("twotemp_1e9", n_lines=240_000, n_chunks=4, n_states=100_000)
    sizes = wl.chunk_sizes()
    assert len(sizes) == 4 and len(wl.conditions) == 4
    ds = P.DeviceStates.from_numpy(wl.states)
    plan = make_plan(wl, prec, max(sizes))
    nb = wl.grid.n_bins
    streamed = torch.zeros((4, nb), dtype=torch.float64, device="cuda")
    st = P.ChunkStreamer(plan, max(sizes))
    n = st.run(ds, wl.chunks(), streamed)
    assert n == sum(sizes)
    resident = torch.zeros_like(streamed)
    for j in range(wl.n_chunks):
        dl = P.DeviceLines.from_numpy(wl.chunk(j))
        plan.cross_section(ds, dl, out=resident, accumulate=j > 0)
    torch.cuda.synchronize()
    assert torch.equal(streamed, resident)
    whole = wl.lines()
    bins = synth.sample_bins(nb, 4000, 3)
    got_all = streamed.cpu().numpy()
    for c, cond in enumerate(wl.conditions):
        r0 = oracle.run_condition(wl, whole, cond, with_sigma=False)
        top = np.argsort(np.abs(r0.S))[-200:]
        kc = np.rint((r0.nu[top] - wl.grid.nu0) / wl.grid.dnu).astype(np.int64)
        near = (kc[:, None] + np.arange(-4, 5)[None, :]).ravel()
        near = near[(near >= 0) & (near < nb)]
        b = np.unique(np.concatenate([bins, near, [int(np.argmax(got_all[c]))]]))
        ref = oracle.run_condition(wl, whole, cond, bins=b).sigma
        e, l1, m = rel_err(got_all[c][b], ref)
        log(f"[stream] prec={prec} Tv={cond.T_vib} Tr={cond.T_rot}: max_rel={e:.2e} L1={l1:.2e} points={m}")
        assert m > 200
        assert e <= (1e-10 if prec == FP64 else 1e-4)
    plan.close()
