"""Shared runner of the end-to-end GPU parity cases (no method arithmetic).

run_case calls the fused end-to-end entry point and the three stages on the
same weights and checks that they agree bit for bit; it can also check which
map kernel the fused call launched (the library's per-launch profile names
the kinds), so that a test can pin the code path it means to cover.
check_against_oracle compares the result with the CPU oracle.
"""
import numpy as np

import oracle
from parity_util import assert_monotone_unit, classify_mismatches

# binary32 spacings: the device and host logf are each within 1 ulp of the
# exact value, so |dz_i| <= 2^-22 z_i, |dZ_i| <= 2^-22 Z_i and
# |du_i| <= 2^-21 u_i.
DU_FP32 = 2.0**-21
DU_FP64 = 1e-12
DW_CAP = 2.0**-40


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def profiled(dcr, fn):
    """Runs fn() with per-launch timing on; returns (fn's result, launch
    counts by kind)."""
    dcr.dcr_profile_begin(64)
    try:
        res = fn()
    finally:
        prof = dcr.dcr_profile_end()
    return res, {k: v[0] for k, v in prof.items() if v[0] > 0}


def run_case(dcr, dev, w, N, seed, stream, expect=None):
    """Fused call (with and without W and u outputs) against the staged calls.

    expect: a launch kind ("finish", "map_fused", "map_dense", ...) that the
    fused call must have launched.
    """
    import torch
    M = w.shape[0]
    wt = to_dev(w, dev)
    W = torch.empty(M, dtype=torch.float64, device=dev)
    u = torch.empty(max(N, 1), dtype=torch.float64, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    r, kinds = profiled(dcr, lambda: dcr.dcr_resample(wt, N, seed, stream, W_out=W, u_out=u,
                                                      dev_status=st))
    if expect is not None:
        assert kinds.get(expect, 0) == 1, f"expected one {expect} launch, got {kinds}"
    r_plain = dcr.dcr_resample(wt, N, seed, stream)        # W and u never written
    W1 = dcr.dcr_cumulative_weights(wt)
    prec = dcr.precision_of(wt)
    u2 = dcr.dcr_sorted_uniforms(N, seed, stream, precision=prec, device=dev)
    r3 = dcr.dcr_inverse_cmf(W1, u2)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    out = dict(r=r.cpu().numpy(), W=W.cpu().numpy(), u=u[:N].cpu().numpy(),
               r_plain=r_plain.cpu().numpy(), W1=W1.cpu().numpy(), u2=u2.cpu().numpy(),
               r3=r3.cpu().numpy(), kinds=kinds)
    del wt, W, u, W1, u2
    # fused == staged, bit for bit
    assert np.array_equal(out["r"], out["r_plain"])
    assert np.array_equal(out["W"], out["W1"])
    assert np.array_equal(out["u"], out["u2"])
    assert np.array_equal(out["r"], out["r3"])
    return out


def check_against_oracle(out, w, N, seed, stream, du_cap, dW_cap=DW_CAP, zkind=None):
    r_o, W_o, u_o = oracle.resample(w, N, seed, stream, zkind=zkind)
    assert_monotone_unit(out["W"])
    if N:
        assert np.all(np.diff(out["u"]) >= 0) and out["u"][0] > 0 and out["u"][-1] <= 1
        assert np.all(np.diff(out["r"]) >= 0)
        # the index map is exact on the GPU's own W and u
        r_exact, _ = oracle.dac(out["W"], out["u"])
        assert np.array_equal(out["r"], r_exact)
    dW = np.max(np.abs(out["W"] - W_o))
    du = np.max(np.abs(out["u"] - u_o)) if N else 0.0
    assert dW <= dW_cap, dW
    assert du <= du_cap, du
    n_mis, bad = classify_mismatches(out["r"], r_o, out["u"], u_o, out["W"], W_o)
    assert not bad, f"{len(bad)} mismatches away from bin edges, e.g. {bad[:5]}"
    print(f"  M={len(w)} N={N} dW={dW:.2e} du={du:.2e} bin-edge mismatches={n_mis} "
          f"launches={out.get('kinds')}", flush=True)
    return n_mis
