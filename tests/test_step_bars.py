"""The per-step bars of the mixed-precision GPU tests are sharp enough to matter.

A small numpy model of an FP32 smearing kernel (decoded storage values, FP32 arithmetic,
one rounding per store) must pass the bars of tests/step_bars.py, and each plausible
precision mistake -- the hops rounded to storage one by one, alpha and beta carried in
bf16, the result accumulated in half -- must fail them.  The kernel model here is test
infrastructure written from the storage-format description; it is not the library's code.
"""
import numpy as np
import pytest

from tests import packed
from tests.step_bars import CASES, Model, abs1, codes, inputs, reals, round_and_bar

_AXIS = {0: 2, 1: 1, 2: 0}


def fp32_step(model, t, psi_s, mistake=None):
    """One step in complex64 arithmetic from storage values, rounded to storage."""
    f = np.complex64
    p = psi_s.astype(f)
    hop = 1 if model.one else 2
    acc = np.zeros_like(p)
    for mu in range(3):
        W = model.Wm[t][..., mu, :, :].astype(f)
        fwd = np.einsum('...ab,...b->...a', W, np.roll(p, -hop, axis=_AXIS[mu]))
        bwd = np.einsum('...ba,...b->...a', np.conj(np.roll(W, hop, axis=_AXIS[mu])), np.roll(p, hop, axis=_AXIS[mu]))
        if mistake == "hop_rounding":
            fwd = packed.storage_round_vectors(fwd.astype(np.complex128), model.vprec).astype(f)
            bwd = packed.storage_round_vectors(bwd.astype(np.complex128), model.vprec).astype(f)
        acc = acc + fwd + bwd
    al, be = np.float32(model.alpha), np.float32(model.beta)
    if mistake == "bf16_coefficients":
        al = np.float32(packed.storage_round_vectors(np.full((1, 3), model.alpha, np.complex128), "bf16")[0, 0].real)
        be = np.float32(packed.storage_round_vectors(np.full((1, 3), model.beta, np.complex128), "bf16")[0, 0].real)
    out = al * p + be * acc
    if mistake == "half_accumulation":
        out = out.real.astype(np.float16).astype(np.float32) + 1j * out.imag.astype(np.float16).astype(np.float32)
    return packed.storage_round_vectors(out.astype(np.complex128), model.vprec)


def check(model, t, psi_s, got):
    E = model.err_bound(t, abs1(psi_s))
    m, bar = round_and_bar(model.step(t, psi_s), E, model.vprec)
    diff = np.abs(reals(got) - reals(m))
    within = bool(np.all(diff <= bar))
    frac = 1.0 if model.vprec == "f32" else float(np.mean(codes(got, model.vprec) == codes(m, model.vprec)))
    return within and frac >= 0.99


@pytest.fixture(scope="module")
def case_inputs():
    L, ts = CASES[0]
    return L, ts, inputs(L, ts, 0)


@pytest.mark.parametrize("form", ["f32", "f16s", "bf16", "bf16-w12", "f16s-onelink"])
@pytest.mark.parametrize("mistake", [None, "hop_rounding", "bf16_coefficients", "half_accumulation"])
def test_bars_accept_fp32_and_reject_mistakes(orc, case_inputs, form, mistake):
    L, ts, (U, psi) = case_inputs
    model = Model(orc, U, form)
    if mistake == "hop_rounding" and model.vprec == "f32":
        pytest.skip("rounding a hop to FP32 storage is FP32 arithmetic")
    t = ts[0]
    psi_s = packed.storage_round_vectors(psi[0], model.vprec)
    ok = check(model, t, psi_s, fp32_step(model, t, psi_s, mistake))
    assert ok == (mistake is None)


def test_link_model_rounds_once(orc):
    """The format model rounds each stored real once (to nearest, within half a spacing of the
    format at the entry's size), and rebuilds the third row of SU(3) two-links exactly in FP64."""
    from paper_2301_05518_amd import synth
    L = (4, 3, 5, 1)
    W = orc.build_twolinks(synth.gauge_field(L, "haar", 17))
    re = lambda z: np.stack([z.real, z.imag], -1)
    assert np.abs(packed.storage_round_links(W, "f64-w12") - W).max() < 1e-14
    for prec, fmt in [("f32", "f32"), ("bf16", "bf16")]:
        d = np.abs(re(packed.storage_round_links(W, prec)) - re(W))
        assert np.all(d <= 0.5 * packed.ulp(re(W), fmt) * (1 + 2.0 ** -16) + 2.0 ** -25)
    # F16S: one scale per matrix, s = max |real|; the entry equal to s is stored exactly
    got = re(packed.storage_round_links(W, "f16s")).reshape(W.shape[:-2] + (18,))
    ref = re(W).reshape(W.shape[:-2] + (18,))
    s = np.abs(ref).max(axis=-1, keepdims=True)
    assert np.all(np.abs(got - ref) <= s * (2.0 ** -12 + 2.0 ** -22))
    assert np.allclose(np.abs(got).max(axis=-1), s[..., 0], rtol=2.0 ** -23, atol=0)
    # sixteen-bit twelve-real rows carry no scale
    rows = re(packed.storage_round_links(W, "bf16-w12"))[..., :2, :, :]
    assert np.array_equal(rows, re(packed.storage_round_links(W, "bf16"))[..., :2, :, :])
