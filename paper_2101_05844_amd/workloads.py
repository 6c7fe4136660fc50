"""Seeded synthetic workloads for the Active Set dual bound.

This module only draws random numbers and arranges them into the inputs the
bounding problem takes (Sec. 2, problem eq:noncvx_pb): layer weights and
biases, an l_inf input box, objective rows for logit-difference properties
(Sec. 7.3.1: minimise true logit minus target logit), and the random draws
that decide which ReLUs a branch-and-bound subdomain fixes.  It holds none of
the bounding method's arithmetic, imports nothing from the rest of the
package, and is shared by the GPU path, the tests and the benchmark.

The networks stand in for the paper's trained CIFAR-10/MNIST models (Table 1
"Wide" architecture; the MNIST MLP shape of App. G), which are not available:
weights are N(0, 1/fan_in), biases N(0, 0.1) (second argument = variance),
inputs U[0,1] images with an l_inf ball of radius eps clipped to [0, 1].

Random draws happen in a fixed order: layer by layer (W then b), then the
input centre, then the property, then the subdomain fixes.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# Layer specifications
# ----------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class DenseSpec:
    n_in: int
    n_out: int


@dataclasses.dataclass(frozen=True)
class ConvSpec:
    c_in: int
    h_in: int
    w_in: int
    c_out: int
    k: int
    stride: int
    pad: int

    @property
    def h_out(self) -> int:
        return (self.h_in + 2 * self.pad - self.k) // self.stride + 1

    @property
    def w_out(self) -> int:
        return (self.w_in + 2 * self.pad - self.k) // self.stride + 1


def spec_sizes(spec) -> Tuple[int, int, int]:
    """(n_in, n_out, fan_in) of a layer spec; conv neurons ordered (c, y, x)."""
    if isinstance(spec, DenseSpec):
        return spec.n_in, spec.n_out, spec.n_in
    return (spec.c_in * spec.h_in * spec.w_in,
            spec.c_out * spec.h_out * spec.w_out,
            spec.c_in * spec.k * spec.k)


@dataclasses.dataclass
class Layer:
    """One affine layer x_hat_k = W_k x_{k-1} + b_k (conv in (c, y, x) order)."""
    spec: object
    W: np.ndarray  # float32; dense [n_out, n_in], conv [c_out, c_in, k, k]
    b: np.ndarray  # float32; dense [n_out], conv [c_out]

    @property
    def kind(self) -> str:
        return "dense" if isinstance(self.spec, DenseSpec) else "conv"

    @property
    def n_in(self) -> int:
        return spec_sizes(self.spec)[0]

    @property
    def n_out(self) -> int:
        return spec_sizes(self.spec)[1]


@dataclasses.dataclass
class Schedule:
    """Iteration schedule of the solver (Sec. 7.1 hyper-parameters)."""
    bigm_iters: int = 180
    as_iters: int = 500
    add_every: int = 450      # omega: addition period
    add_count: int = 2        # V: consecutive addition iterations per period
    max_masks: int = 7        # K_max: cap on masks per layer
    bigm_lr: Tuple[float, float] = (1e-2, 1e-4)
    as_lr: Tuple[float, float] = (1e-3, 1e-6)
    adam_beta1: float = 0.9
    adam_beta2: float = 0.999
    adam_eps: float = 1e-8


@dataclasses.dataclass
class Workload:
    name: str
    layers: List[Layer]
    l0: np.ndarray            # float32 [S, n0]
    u0: np.ndarray            # float32 [S, n0]
    c: np.ndarray             # float32 [S, n_last] objective rows
    schedule: Schedule
    fix_draws: Optional["FixDraws"] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def S(self) -> int:
        return self.l0.shape[0]

    @property
    def relu_sizes(self) -> List[int]:
        return [L.n_out for L in self.layers[:-1]]


@dataclasses.dataclass
class FixDraws:
    """Random numbers that decide each subdomain's fixed ReLU phases.

    count[s]   number of ReLUs subdomain s fixes (before capping at the number
               of ambiguous ReLUs);
    key[s, r]  uniform key per ReLU r (flattened over layers); the fixed ReLUs
               are the `count[s]` ambiguous ones with the smallest keys;
    phase[s,r] 1 = passing (pre-activation lower bound raised to 0),
               0 = blocking (pre-activation upper bound lowered to 0).
    """
    count: np.ndarray
    key: np.ndarray
    phase: np.ndarray


# ----------------------------------------------------------------------------
# Drawing
# ----------------------------------------------------------------------------


def draw_layers(specs: Sequence, rng: np.random.Generator) -> List[Layer]:
    layers = []
    for sp in specs:
        _, _, fan_in = spec_sizes(sp)
        if isinstance(sp, DenseSpec):
            W = rng.normal(0.0, np.sqrt(1.0 / fan_in), size=(sp.n_out, sp.n_in))
            b = rng.normal(0.0, np.sqrt(0.1), size=(sp.n_out,))
        else:
            W = rng.normal(0.0, np.sqrt(1.0 / fan_in),
                           size=(sp.c_out, sp.c_in, sp.k, sp.k))
            b = rng.normal(0.0, np.sqrt(0.1), size=(sp.c_out,))
        layers.append(Layer(sp, W.astype(np.float32), b.astype(np.float32)))
    return layers


def linf_box(centre: np.ndarray, eps: float, clip: Optional[Tuple[float, float]]):
    lo = centre - eps
    hi = centre + eps
    if clip is not None:
        lo = np.clip(lo, clip[0], clip[1])
        hi = np.clip(hi, clip[0], clip[1])
    return lo.astype(np.float32), hi.astype(np.float32)


def logit_difference_rows(n_classes: int, true_cls: int, targets: Sequence[int]) -> np.ndarray:
    """Objective rows c = e_true - e_target (minimise true minus target logit)."""
    c = np.zeros((len(targets), n_classes), dtype=np.float32)
    for r, j in enumerate(targets):
        c[r, true_cls] = 1.0
        c[r, j] = -1.0
    return c


def draw_fixes(rng: np.random.Generator, S: int, n_relu: int, max_count: int) -> FixDraws:
    count = rng.integers(0, max_count + 1, size=S)
    key = rng.random((S, n_relu))
    phase = rng.integers(0, 2, size=(S, n_relu)).astype(np.int8)
    return FixDraws(count=count, key=key, phase=phase)


def select_fixes(draws: FixDraws, ambiguous: np.ndarray, s: int):
    """Indices (into the flattened ReLU list) and phases fixed by subdomain s.

    `ambiguous` is a boolean vector over all ReLUs (flattened over layers)
    marking those whose pre-activation interval strictly contains 0 at the
    root.  Pure selection: no bound arithmetic.
    """
    cand = np.flatnonzero(ambiguous)
    n = min(int(draws.count[s]), cand.size)
    if n == 0:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int8)
    order = np.argsort(draws.key[s, cand], kind="stable")[:n]
    idx = np.sort(cand[order])
    return idx, draws.phase[s, idx]


def subdomain_bounds(root_lhat: Sequence[np.ndarray], root_uhat: Sequence[np.ndarray],
                     draws: Optional[FixDraws], S: int):
    """Per-subdomain pre-activation bounds [S, n_k] from root bounds.

    Root bounds are [n_k] (one root shared by all subdomains) or [S, n_k]
    (one root per subproblem).  A branch-and-bound split fixes a ReLU's phase:
    passing sets the lower pre-activation bound to 0, blocking sets the upper
    one to 0 (Sec. 7.3: BaBSR splits a ReLU into its two phases).  The other
    bounds stay as they are at the root, which remains valid on the subdomain.
    """
    def per_s(a):
        a = np.asarray(a, np.float32)
        return np.repeat(a[None, :], S, axis=0) if a.ndim == 1 else a.copy()

    lh = [per_s(a) for a in root_lhat]
    uh = [per_s(a) for a in root_uhat]
    if draws is None:
        return lh, uh
    offs = np.cumsum([0] + [a.shape[1] for a in lh])
    for s in range(S):
        flat_l = np.concatenate([a[s] for a in lh])
        flat_u = np.concatenate([a[s] for a in uh])
        ambiguous = (flat_l < 0) & (flat_u > 0)
        idx, ph = select_fixes(draws, ambiguous, s)
        for r, p in zip(idx, ph):
            k = int(np.searchsorted(offs, r, side="right") - 1)
            i = int(r - offs[k])
            if p:
                lh[k][s, i] = 0.0
            else:
                uh[k][s, i] = 0.0
    return lh, uh


# ----------------------------------------------------------------------------
# The configurations
# ----------------------------------------------------------------------------

TINY_SPECS = [DenseSpec(5, 8), DenseSpec(8, 8), DenseSpec(8, 1)]
MNIST_SPECS = [DenseSpec(784, 100), DenseSpec(100, 100), DenseSpec(100, 100), DenseSpec(100, 10)]
CIFAR_WIDE_SPECS = [
    ConvSpec(3, 32, 32, 16, 4, 2, 1),
    ConvSpec(16, 16, 16, 32, 4, 2, 1),
    DenseSpec(2048, 100),
    DenseSpec(100, 10),
]
CIFAR_WIDER_SPECS = [
    ConvSpec(3, 32, 32, 32, 4, 2, 1),
    ConvSpec(32, 16, 16, 64, 4, 2, 1),
    DenseSpec(4096, 512),
    DenseSpec(512, 10),
]


def tiny_config(seed: int = 1000) -> Workload:
    """5-8-8-1 ReLU net, box centre U[-1,1]^5 +- 0.1, one subproblem."""
    rng = np.random.default_rng(seed)
    layers = draw_layers(TINY_SPECS, rng)
    centre = rng.uniform(-1.0, 1.0, size=5)
    l0, u0 = linf_box(centre, 0.1, None)
    c = np.ones((1, 1), dtype=np.float32)
    sched = Schedule(bigm_iters=50, as_iters=50, add_every=10, add_count=2, max_masks=7)
    return Workload("tiny-5-8-8-1", layers, l0[None, :], u0[None, :], c, sched,
                    meta={"seed": seed, "eps": 0.1})


def mnist_mlp_config(seed: int = 1001) -> Workload:
    """784-100-100-100-10 MLP, eps 0.05, 9 logit-difference subproblems."""
    rng = np.random.default_rng(seed)
    layers = draw_layers(MNIST_SPECS, rng)
    centre = rng.uniform(0.0, 1.0, size=784)
    eps = 0.05
    l0, u0 = linf_box(centre, eps, (0.0, 1.0))
    t = int(rng.integers(0, 10))
    targets = [j for j in range(10) if j != t]
    c = logit_difference_rows(10, t, targets)
    S = len(targets)
    sched = Schedule(bigm_iters=500, as_iters=500, add_every=450, add_count=2, max_masks=7,
                     bigm_lr=(1e-1, 1e-3), as_lr=(1e-3, 1e-6))
    return Workload("mnist-mlp-784-100x3-10", layers, np.repeat(l0[None], S, 0),
                    np.repeat(u0[None], S, 0), c, sched,
                    meta={"seed": seed, "eps": eps, "true_class": t})


def cifar_conv_config(seed: int = 1002, S: int = 512, specs=None, max_fixed: int = 20,
                      name: str = "cifar-wide-conv") -> Workload:
    """Table 1 "Wide" CIFAR conv net, eps 2/255, S branch-and-bound subdomains.

    All subdomains share one input box and one property; each fixes
    U{0..max_fixed} ambiguous ReLUs (drawn for 512 subdomains, so smaller S
    takes a prefix of the same draws).
    """
    specs = CIFAR_WIDE_SPECS if specs is None else specs
    rng = np.random.default_rng(seed)
    layers = draw_layers(specs, rng)
    centre = rng.uniform(0.0, 1.0, size=3 * 32 * 32)
    eps = 2.0 / 255.0
    l0, u0 = linf_box(centre, eps, (0.0, 1.0))
    t = int(rng.integers(0, 10))
    j = int(rng.choice([k for k in range(10) if k != t]))
    c = logit_difference_rows(10, t, [j])
    n_relu = sum(spec_sizes(sp)[1] for sp in specs[:-1])
    S_draw = max(512, S)
    draws = draw_fixes(rng, S_draw, n_relu, max_fixed)
    draws = FixDraws(draws.count[:S], draws.key[:S], draws.phase[:S])
    sched = Schedule(bigm_iters=180, as_iters=500, add_every=450, add_count=2, max_masks=7)
    return Workload(name, layers, np.repeat(l0[None], S, 0), np.repeat(u0[None], S, 0),
                    np.repeat(c, S, 0), sched, fix_draws=draws,
                    meta={"seed": seed, "eps": eps, "true_class": t, "target": j})


def network_output(layers: Sequence[Layer], x0: np.ndarray) -> np.ndarray:
    """Plain forward pass of the network (FP64) at one input: picks the
    property of a workload, outside the method."""
    x = np.asarray(x0, dtype=np.float64)
    for i, L in enumerate(layers):
        if L.kind == "dense":
            y = L.W.astype(np.float64) @ x.reshape(-1) + L.b
        else:
            sp = L.spec
            xin = x.reshape(sp.c_in, sp.h_in, sp.w_in)
            xp = np.pad(xin, ((0, 0), (sp.pad, sp.pad), (sp.pad, sp.pad)))
            y = np.zeros((sp.c_out, sp.h_out, sp.w_out))
            W = L.W.astype(np.float64).reshape(sp.c_out, sp.c_in, sp.k, sp.k)
            for ky in range(sp.k):
                for kx in range(sp.k):
                    patch = xp[:, ky:ky + sp.stride * sp.h_out:sp.stride, kx:kx + sp.stride * sp.w_out:sp.stride]
                    y += np.einsum("oc,chw->ohw", W[:, :, ky, kx], patch)
            y += L.b.astype(np.float64)[:, None, None]
            y = y.reshape(-1)
        x = np.maximum(y, 0.0) if i + 1 < len(layers) else y
    return x


def cifar_margin_config(seed: int = 1006, S: int = 512, eps: float = 0.5 / 255.0, max_fixed: int = 20,
                        net_seed: int = 1002) -> Workload:
    """Accuracy workload on the CIFAR "Wide" net of cifar_conv_config (same
    weights): a centre U[0,1]^3072 whose top class t under the network is
    the true class, a smaller radius eps (so that part of the subdomains can
    be verified, bound > 0), and S branch-and-bound subdomains fixing
    U{0..max_fixed} ambiguous ReLUs each; subdomain s bounds the logit
    difference of t against the (1 + s mod 9)-th class by output, so the
    margins at the centre span easy and hard properties."""
    layers = draw_layers(CIFAR_WIDE_SPECS, np.random.default_rng(net_seed))
    rng = np.random.default_rng(seed)
    centre = rng.uniform(0.0, 1.0, size=3 * 32 * 32)
    out = network_output(layers, centre)
    order = np.argsort(-out)
    t = int(order[0])
    targets = [int(order[1 + s % 9]) for s in range(S)]
    l0, u0 = linf_box(centre, eps, (0.0, 1.0))
    c = np.concatenate([logit_difference_rows(10, t, [j]) for j in targets], axis=0)
    n_relu = sum(spec_sizes(sp)[1] for sp in CIFAR_WIDE_SPECS[:-1])
    draws = draw_fixes(rng, S, n_relu, max_fixed)
    sched = Schedule(bigm_iters=180, as_iters=500, add_every=450, add_count=2, max_masks=7)
    return Workload("cifar-wide-margin", layers, np.repeat(l0[None], S, 0), np.repeat(u0[None], S, 0),
                    c, sched, fix_draws=draws,
                    meta={"seed": seed, "net_seed": net_seed, "eps": eps, "true_class": t,
                          "margins_at_centre": [float(out[t] - out[int(order[1 + i])]) for i in range(9)]})


def adjoint_config(seed: int = 1004, n_inputs: int = 256, net_seed: int = 1002) -> Workload:
    """Bound-gradient workload: the CIFAR "Wide" net of cifar_conv_config
    (same weights), n_inputs centres U[0,1]^3072 with eps 2/255 clipped to
    [0, 1], and for each input its 9 logit differences (true class from the
    seed): S = 9 n_inputs root subproblems, input-major.  Pre-activation
    bounds come from interval propagation per input (no fixed ReLUs)."""
    layers = draw_layers(CIFAR_WIDE_SPECS, np.random.default_rng(net_seed))
    rng = np.random.default_rng(seed)
    centre = rng.uniform(0.0, 1.0, size=(n_inputs, 3 * 32 * 32))
    eps = 2.0 / 255.0
    l0, u0 = linf_box(centre, eps, (0.0, 1.0))
    true = rng.integers(0, 10, size=n_inputs)
    rows = [logit_difference_rows(10, int(t), [j for j in range(10) if j != t]) for t in true]
    c = np.concatenate(rows, axis=0)
    sched = Schedule(bigm_iters=180, as_iters=500, add_every=450, add_count=2, max_masks=7)
    return Workload("cifar-wide-adjoint", layers, np.repeat(l0, 9, 0), np.repeat(u0, 9, 0), c, sched,
                    meta={"seed": seed, "net_seed": net_seed, "eps": eps, "centre": centre.astype(np.float32),
                          "true_class": true})


def ragged_config(seed: int = 1003, S: int = 4096, net_seeds=(1002, 1005), max_fixed: int = 50,
                  budget_range=(100, 1000)):
    """Ragged batch of branch-and-bound subdomains: S/2 on the CIFAR "Wide"
    net of cifar_conv_config (same weights) and S/2 on its wider variant
    (conv 3->32 and 32->64, FC 4096->512->10), one input box and property
    per net (3x32x32 U[0,1], eps 2/255), each subdomain fixing U{0..max_fixed}
    ambiguous ReLUs and carrying its own Active Set budget U{budget_range}.
    Returns one Workload per net (subdomains ordered by non-increasing
    budget, budgets in meta["budgets"])."""
    rng = np.random.default_rng(seed)
    out = []
    for i, (specs, nseed) in enumerate(((CIFAR_WIDE_SPECS, net_seeds[0]), (CIFAR_WIDER_SPECS, net_seeds[1]))):
        layers = draw_layers(specs, np.random.default_rng(nseed))
        Sn = S // 2 if i == 0 else S - S // 2
        centre = rng.uniform(0.0, 1.0, size=3 * 32 * 32)
        eps = 2.0 / 255.0
        l0, u0 = linf_box(centre, eps, (0.0, 1.0))
        t = int(rng.integers(0, 10))
        j = int(rng.choice([k for k in range(10) if k != t]))
        c = logit_difference_rows(10, t, [j])
        n_relu = sum(spec_sizes(sp)[1] for sp in specs[:-1])
        draws = draw_fixes(rng, Sn, n_relu, max_fixed)
        budgets = np.sort(rng.integers(budget_range[0], budget_range[1] + 1, size=Sn))[::-1].copy()
        sched = Schedule(bigm_iters=180, as_iters=int(budgets[0]), add_every=450, add_count=2, max_masks=7)
        out.append(Workload(f"ragged-{'wide' if i == 0 else 'wider'}", layers, np.repeat(l0[None], Sn, 0),
                            np.repeat(u0[None], Sn, 0), np.repeat(c, Sn, 0), sched, fix_draws=draws,
                            meta={"seed": seed, "net_seed": nseed, "eps": eps, "true_class": t, "target": j,
                                  "budgets": [int(b) for b in budgets]}))
    return out


def custom_config(specs: Sequence, S: int, seed: int, eps: float = 0.05,
                  centre_range=(0.0, 1.0), n_props: Optional[int] = None,
                  max_fixed: int = 0, schedule: Optional[Schedule] = None,
                  name: str = "custom") -> Workload:
    """Arbitrary small net for parity tests (ragged sizes, several tiles).

    Each subproblem gets its own random objective row (N(0,1) entries) unless
    the last layer has one output, in which case c = 1.
    """
    rng = np.random.default_rng(seed)
    layers = draw_layers(specs, rng)
    n0 = layers[0].n_in
    centre = rng.uniform(centre_range[0], centre_range[1], size=(S, n0))
    clip = (0.0, 1.0) if centre_range == (0.0, 1.0) else None
    l0, u0 = linf_box(centre, eps, clip)
    n_last = layers[-1].n_out
    if n_last == 1:
        c = np.ones((S, 1), dtype=np.float32)
    else:
        c = rng.normal(0.0, 1.0, size=(S, n_last)).astype(np.float32)
    draws = None
    if max_fixed > 0:
        n_relu = sum(L.n_out for L in layers[:-1])
        draws = draw_fixes(rng, S, n_relu, max_fixed)
    sched = schedule or Schedule(bigm_iters=20, as_iters=30, add_every=10, add_count=2,
                                 max_masks=3)
    return Workload(name, layers, l0, u0, c, sched, fix_draws=draws,
                    meta={"seed": seed, "eps": eps})


def make_config(i: int, S: Optional[int] = None) -> Workload:
    """Configurations by index: 0 tiny, 1 MNIST MLP, 2 CIFAR conv (S default 512)."""
    if i == 0:
        return tiny_config()
    if i == 1:
        return mnist_mlp_config()
    if i == 2:
        return cifar_conv_config(S=512 if S is None else S)
    raise ValueError(f"unknown configuration {i}")


def random_points_in_box(l0: np.ndarray, u0: np.ndarray, n: int, seed: int) -> np.ndarray:
    """n uniform points and the 2 extreme corners of a box [n0] (for sampled outputs)."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, size=(n, l0.shape[0]))
    pts = l0[None, :] + pts * (u0 - l0)[None, :]
    return np.concatenate([pts, l0[None, :], u0[None, :]], axis=0)
