"""Per-step arithmetic of the mixed-precision storage forms, through the C ABI.

One or two smearing steps (eq. tlSmear) of every 32- and 16-bit storage form are
compared with an expectation built only from the oracle and the test-side format
model (tests/packed.py): the FP64 step of the oracle applied to the inputs as the
format stores them (colour vectors and links rounded by the model, never read back
from the GPU), its result rounded by the same model.  The kernels compute in FP32 from
exactly decoded storage values and round once per store, so a kernel result may differ
from that expectation only through FP32 arithmetic, bounded per real component by

    E = u32 (40 A + 16 B)

where A is the step evaluated on absolute values (|alpha| |psi| + beta sum_hops |W| |psi|,
|z| = |re| + |im|): a real output component is a sum of 37 products (alpha psi and six
3x3 complex mat-vecs), so at most about 38 roundings plus the FP32 rounding of alpha and
beta, 40 u32 A in all; B (twelve-real links only) is beta sum_hops sum_c |psi_c|, which
with the 16 u32 bound on a rebuilt third-row entry covers the FP32 cross product.
The storage rounding turns E into:

* FP32: |gpu - model| <= E + ulp32
* BF16: |gpu - model| <= E + ulp_bf16 + ulp32  (both sides round once to bf16)
* F16S: |gpu - model| <= s ulp_half(q) + 3 (E_site + ulp32(s)) + 4 u32 s, with s the
  site's scale (max |real|) and q = value / s: the half codes can differ by one where the
  two results straddle a rounding boundary, and the scales by the FP32 error.

The 16-bit forms must also store the model's code (bf16 bits, or half code of value / s)
in at least 99% of the components after one step and 98% after two: a code differs only
where the FP32 error E straddles a rounding boundary, a fraction of about E / ulp_storage
(well below 1%).  Rounding per hop, alpha or beta carried in 16 bits, or 16-bit
accumulation move whole fractions of an ulp and fail these counts; FP32 results fail
the E bound by orders of magnitude.  For two steps the first step's difference bound D is
propagated through the second by the same absolute-value step (|alpha| D + beta sum |W| D)
and added to E.
"""
import numpy as np
import pytest

from paper_2301_05518_amd import synth
from tests import packed
from tests.gpu_common import log, to_dev
from tests.step_bars import CASES, FORMS, TILES, Model, abs1, codes, inputs, reals, round_and_bar, split

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2301_05518_amd as tl
    c = tl.Context(0)
    yield c
    c.close()


def gpu_run(ctx, torch, L, U, ts, psi, form, n, sigma, tile, monkeypatch):
    import paper_2301_05518_amd as tl
    monkeypatch.setenv("TL_TILE", tile)
    links, _, one = split(form)
    Ud = to_dev(U)
    W = ctx.pack_links(L, Ud, form) if one else ctx.build_twolinks(L, Ud, form)
    jobs = [tl.Job(tuple(L), W, list(ts), to_dev(psi))]
    ctx.smear(jobs, n, sigma, form)
    torch.cuda.synchronize()
    return jobs[0].psi.cpu().numpy()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[str(c[0]) for c in CASES])
@pytest.mark.parametrize("form", FORMS)
def test_one_and_two_steps(ctx, orc, torch, form, case, monkeypatch):
    L, ts = CASES[case]
    U, psi = inputs(L, ts, case)
    model = Model(orc, U, form)
    vprec = model.vprec
    psi_s = packed.storage_round_vectors(psi, vprec)   # what the pack stores
    for n in (1, 2):
        sigma = n * model.s
        outs = [gpu_run(ctx, torch, L, U, ts, psi, form, n, sigma, tile, monkeypatch) for tile in TILES]
        assert np.array_equal(outs[0], outs[1]), "tilings disagree"
        gpu = outs[0]
        worst, match = 0.0, []
        for r, t in enumerate(ts):
            cur = psi_s[r]
            D = np.zeros(cur.shape)          # bound on |gpu - model| of the step's input, per colour (|.|_1)
            for k in range(n):
                d = abs1(cur) + D
                E = model.err_bound(t, d.astype(np.complex128)) + model.propagate(t, D)
                m, bar = round_and_bar(model.step(t, cur), E, vprec)
                if k == n - 1:
                    diff = np.abs(reals(gpu[r]) - reals(m))
                    worst = max(worst, float(np.max(diff / bar)))
                    assert np.all(diff <= bar), (r, k, float(np.max(diff / bar)))
                    if vprec != "f32":
                        match.append(codes(gpu[r], vprec) == codes(m, vprec))
                D = 2.0 * np.max(bar, axis=-1)   # |.|_1 of a complex difference <= 2 max(re, im)
                cur = m
        frac = float(np.mean(np.concatenate([x.ravel() for x in match]))) if match else 1.0
        log(f"{form} {L} n={n}: worst |gpu - model| / bar = {worst:.3f}, codes equal {frac:.5f}")
        if vprec != "f32":
            assert frac >= (0.99 if n == 1 else 0.98), frac


@pytest.mark.parametrize("form", ["f32", "f16s", "bf16", "f16s-w12", "bf16-w12"])
def test_link_model_matches_stored_links(ctx, orc, torch, form):
    """The format model's links are the library's stored links (decoded by the test-side reader)."""
    L = (12, 10, 9, 2)
    U = synth.gauge_field(L, "haar", 5399)
    got = packed.decode_twolinks(ctx.build_twolinks(L, to_dev(U), form).cpu().numpy(), L, form, L[3])
    want = packed.storage_round_links(orc.build_twolinks(U), form)
    rows = 2 if form.endswith("-w12") else 3
    g, w = got[..., :rows, :], want[..., :rows, :]
    same = float(np.mean((g.real == w.real) & (g.imag == w.imag)))
    log(f"{form}: stored links equal to the model in {same:.6f} of the entries")
    # the library's FP64 product may differ from the oracle's in the last bit, which moves a
    # rounding only where the product sits on a boundary of the storage format
    assert same >= 0.9999
    spacing = {"f32": 2.0 ** -24, "f16s": 2.0 ** -11, "bf16": 2.0 ** -8}[form.replace("-w12", "")]
    assert np.max(np.abs(g - w)) <= 2 * spacing
