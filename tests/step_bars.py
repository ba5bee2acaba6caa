"""Per-step expectation and bars of the mixed-precision storage forms (see
tests/test_gpu_step_rounding.py for the derivation): the oracle's FP64 step on
storage-rounded inputs, the model rounding of its result, and the FP32 error bound."""
import numpy as np

from paper_2301_05518_amd import synth
from tests import packed

U32 = 2.0 ** -24
FORMS = ["f32", "f16s", "bf16", "f32-w12", "f16s-w12", "bf16-w12", "f32-onelink", "f16s-onelink", "bf16-onelink"]
# (shape, slice of every RHS): a ragged one (groups of 3 and 1 RHS) and one with rows of
# 64 sites, where the LDS kernels take the backward x link from the neighbouring lane
CASES = [((12, 10, 9, 2), [1, 1, 0, 1]), ((64, 8, 6, 1), [0, 0, 0])]
# default direct kernel, and the pipelined LDS kernel in the benchmark's tiling
TILES = ["0,256,4,0", "7,512,16,0,1,1"]
STEP = {"two": 0.4, "one": 0.1}    # sigma / n: alpha = 0.4, beta = 0.1 for both operators


def split(form):
    one = form.endswith("-onelink")
    links = form[:-8] if one else form
    return links, links.replace("-w12", ""), one


def inputs(L, ts, seed):
    U = synth.gauge_field(L, "haar", 5300 + seed)
    rng = np.random.default_rng([5301, seed])
    psi = synth.random_field(rng, (len(ts), L[2], L[1], L[0], 3))
    # per-site magnitudes over four decades: varied F16S scales, and hops that cancel
    psi *= np.exp2(rng.uniform(-6.0, 6.0, size=psi.shape[:-1]))[..., None]
    return U, psi


def abs1(z):
    """|re| + |im| as a complex array with zero imaginary part."""
    return (np.abs(z.real) + np.abs(z.imag)).astype(np.complex128)


class Model:
    """The oracle's FP64 step on storage-rounded links, and its absolute-value companion."""

    def __init__(self, orc, U, form):
        self.orc = orc
        self.links, self.vprec, self.one = split(form)
        s = STEP["one" if self.one else "two"]
        self.s = s
        self.alpha = 1.0 - 6.0 * (s if self.one else 0.25 * s)
        self.beta = s if self.one else 0.25 * s
        if self.one:
            Ur = U.copy()
            Ur[..., :3, :, :] = packed.storage_round_links(U[..., :3, :, :], self.links)
            self.Wm = Ur
            self.Wabs = abs1(Ur)
            J = np.zeros_like(Ur)
            J[..., :3, :, :] = 1.0
        else:
            self.Wm = packed.storage_round_links(orc.build_twolinks(U), self.links)
            self.Wabs = abs1(self.Wm)
            J = np.ones_like(self.Wm)
        self.J = J

    def step(self, t, psi):
        """psi + s Lap psi in FP64 (the oracle's literal form of one step)."""
        if self.one:
            return self.orc.smear_onelink(self.Wm, t, 1, self.s, psi)
        return self.orc.smear(self.Wm, t, 1, self.s, psi)

    def hops_abs(self, M, t, d):
        """sum_hops M d for non-negative real M (as complex) and d: 4 Lap + 6 (two-link), Lap + 6 (one-link)."""
        if self.one:
            return (self.orc.laplacian_onelink(M, t, d) + 6.0 * d).real
        return (4.0 * self.orc.laplacian(M, t, d) + 6.0 * d).real

    def err_bound(self, t, d):
        """E per colour (valid for the real and the imaginary part) for inputs with |.|_1 = d."""
        A = abs(self.alpha) * d.real + self.beta * self.hops_abs(self.Wabs, t, d)
        B = self.beta * self.hops_abs(self.J, t, d) if self.links.endswith("-w12") else 0.0
        return U32 * (40.0 * A + 16.0 * B)

    def propagate(self, t, D):
        """|alpha| D + beta sum_hops |W| D: bound on how a difference D of the input moves the output."""
        Dc = D.astype(np.complex128)
        return abs(self.alpha) * D + self.beta * self.hops_abs(self.Wabs, t, Dc)


def reals(z):
    return np.stack([z.real, z.imag], axis=-1)   # [..][3][2]


def round_and_bar(r64, E, vprec):
    """Model rounding of the FP64 step result, and the per-real bar |gpu - model| for FP32 error E."""
    m = packed.storage_round_vectors(r64, vprec)
    R = reals(r64)
    Er = np.repeat(E[..., None], 2, axis=-1)
    if vprec == "f32":
        bar = Er + packed.ulp(np.abs(R) + Er, "f32")
    elif vprec == "bf16":
        bar = Er + packed.ulp(np.abs(R) + Er, "bf16") + packed.ulp(np.abs(R), "f32")
    else:   # f16s: per-site scale
        flat = R.reshape(R.shape[:-2] + (6,))
        s = np.max(np.abs(flat.astype(np.float32)).astype(np.float64), axis=-1)[..., None, None]
        Es = np.max(Er.reshape(Er.shape[:-2] + (6,)), axis=-1)[..., None, None]
        es = Es + packed.ulp(s, "f32")
        ss = np.where(s > 0, s, 1.0)
        q = np.abs(R) / ss + 2.0 * es / ss
        bar = np.where(s > 0, s * packed.ulp(q, "half") + 3.0 * es + 4.0 * U32 * s, Er)
    return m, bar


def codes(v, vprec):
    """Storage codes of decoded values: bf16 values themselves; F16S half codes of value / scale."""
    R = reals(v)
    if vprec == "bf16":
        return R
    flat = R.reshape(R.shape[:-2] + (6,))
    s = np.max(np.abs(flat), axis=-1)[..., None, None]
    return (R / np.where(s > 0, s, 1.0)).astype(np.float16)


