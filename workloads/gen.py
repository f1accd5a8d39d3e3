"""Counter-based, seeded input generators (torch; identical code on CPU and GPU).

Every value is a pure function of (seed, stream, index), so any slice of an
input can be regenerated independently and the same call gives the same bytes
on every run.  Unsigned 64-bit words are carried in torch.int64 tensors as bit
patterns (torch has no full uint64 arithmetic); right shifts are made logical
by masking.

Primitives
----------
* ``mix64``: the splitmix64 output function (Steele, Lea & Flood, "Fast
  splittable pseudorandom number generators", OOPSLA 2014, with Stafford's
  "Mix13" finaliser constants).
* ``rand64(seed, stream, i)``: output i+1 of a splitmix64 sequence whose state
  starts at ``mix64(seed ^ mix64(stream + GOLDEN))``.
* Zipf ranks: rejection-inversion sampling (Hoermann & Derflinger, "Rejection-
  inversion to generate variates from monotone discrete distributions", 1996).
* Rank -> key bijections: 4-round balanced Feistel networks keyed by the seed.

Workloads (the sizes and shapes of the paper's synthetic distributions and of
the five benchmark configurations) are assembled by ``make_config``.
"""
from __future__ import annotations

import math

import torch

GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _s64(c: int) -> int:
    """Unsigned 64-bit constant -> the int64 with the same bit pattern."""
    c &= (1 << 64) - 1
    return c - (1 << 64) if c >= (1 << 63) else c


def _lsr(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def mix64(x: torch.Tensor) -> torch.Tensor:
    z = x
    z = (z ^ _lsr(z, 30)) * _s64(_M1)
    z = (z ^ _lsr(z, 27)) * _s64(_M2)
    return z ^ _lsr(z, 31)


def _mix64_int(x: int) -> int:
    m = (1 << 64) - 1
    z = x & m
    z = ((z ^ (z >> 30)) * _M1) & m
    z = ((z ^ (z >> 27)) * _M2) & m
    return z ^ (z >> 31)


def _base(seed: int, stream: int) -> int:
    return _mix64_int((seed & ((1 << 64) - 1)) ^ _mix64_int(stream + GOLDEN))


def rand64(seed: int, stream: int, n: int, device="cpu", start: int = 0) -> torch.Tensor:
    """n pseudo-random 64-bit words (int64 bit patterns) for indices start..start+n-1."""
    i = torch.arange(start + 1, start + n + 1, dtype=torch.int64, device=device)
    return mix64(i * _s64(GOLDEN) + _s64(_base(seed, stream)))


def uniform01(seed: int, stream: int, n: int, device="cpu", start: int = 0) -> torch.Tensor:
    """Doubles uniform on [0, 1) with 53 random bits."""
    return _lsr(rand64(seed, stream, n, device, start), 11).to(torch.float64) * (2.0 ** -53)


def uniform_u32(n: int, seed: int = 0, device="cpu", stream: int = 1) -> torch.Tensor:
    """Uniform over [0, 2^32): the top 32 bits of each word (int64 values)."""
    return _lsr(rand64(seed, stream, n, device), 32)


def uniform_u64(n: int, seed: int = 0, device="cpu", stream: int = 2) -> torch.Tensor:
    """Uniform over [0, 2^64) (int64 bit patterns)."""
    return rand64(seed, stream, n, device)


def exponential_keys(n: int, lam: float, seed: int = 0, device="cpu", stream: int = 3) -> torch.Tensor:
    """floor(X) with X exponential of rate lam (inverse CDF of 1-U)."""
    u = uniform01(seed, stream, n, device)
    return torch.floor(-torch.log1p(-u) / lam).to(torch.int64)


def bit_exponential_keys(n: int, p: float = 0.1, seed: int = 0, device="cpu", stream: int = 4) -> torch.Tensor:
    """Keys whose significant-bit count k is geometric(p) on {1,2,...} capped at 64,
    with the k-1 bits below the leading one uniform.  int64 bit patterns."""
    u = uniform01(seed, stream, n, device)
    k = 1 + torch.floor(torch.log1p(-u) / math.log1p(-p)).to(torch.int64)
    k = torch.clamp(k, 1, 64)
    low = rand64(seed, stream + 1000, n, device)
    one = torch.ones_like(k)
    lead = torch.bitwise_left_shift(one, k - 1)
    return lead | (low & (lead - 1))


# ---------------------------------------------------------------- Zipf ranks
def _helper1(x):
    small = x.abs() <= 1e-8
    xs = torch.where(small, torch.ones_like(x), x)
    return torch.where(small, 1.0 - x * (0.5 - x * (1.0 / 3.0 - 0.25 * x)), torch.log1p(xs) / xs)


def _helper2(x):
    small = x.abs() <= 1e-8
    xs = torch.where(small, torch.ones_like(x), x)
    return torch.where(small, 1.0 + x * 0.5 * (1.0 + x / 3.0 * (1.0 + 0.25 * x)), torch.expm1(xs) / xs)


def zipf_ranks(n: int, s: float, N, seed: int = 0, device="cpu", stream: int = 5,
               max_rounds: int = 200) -> torch.Tensor:
    """Ranks in 1..N with P(k) proportional to k^-s (rejection-inversion).

    ``N`` may be a Python number or a float64 tensor of length n (one range per element).
    """
    f64 = torch.float64
    if torch.is_tensor(N):
        Nt = N.to(device=device, dtype=f64)
    else:
        Nt = torch.full((n,), float(N), dtype=f64, device=device)
    one_minus_s = 1.0 - s

    def H(x):
        lx = torch.log(x)
        return _helper2(one_minus_s * lx) * lx

    def Hinv(x):
        t = torch.clamp(x * one_minus_s, min=-1.0)
        return torch.exp(_helper1(t) * x)

    def h(x):
        return torch.exp(-s * torch.log(x))

    c = lambda v: torch.full((1,), v, dtype=f64, device=device)
    hx1 = H(c(1.5)) - 1.0
    hN = H(Nt + 0.5)
    s_param = 2.0 - Hinv(H(c(2.5)) - h(c(2.0)))

    out = torch.zeros(n, dtype=torch.int64, device=device)
    pending = torch.arange(n, device=device)
    for r in range(max_rounds):
        if pending.numel() == 0:
            break
        u01 = uniform01(seed, stream * 1024 + r, n, device)[pending]
        hn = hN[pending]
        u = hn + u01 * (hx1 - hn)
        x = Hinv(u)
        k = torch.floor(x + 0.5)
        k = torch.minimum(torch.clamp(k, min=1.0), Nt[pending])
        acc = (k - x <= s_param) | (u >= H(k + 0.5) - h(k))
        out[pending[acc]] = k[acc].to(torch.int64)
        pending = pending[~acc]
    if pending.numel():
        raise RuntimeError("zipf_ranks: rejection sampling did not converge")
    return out


# ---------------------------------------------------------------- bijections
def feistel32(x: torch.Tensor, key: int) -> torch.Tensor:
    """Bijection on [0, 2^32) (values in int64)."""
    L = _lsr(x, 16) & 0xFFFF
    R = x & 0xFFFF
    for r in range(4):
        kr = _s64(_mix64_int(key * 4 + r + GOLDEN))
        F = mix64(R ^ kr) & 0xFFFF
        L, R = R, L ^ F
    return (L << 16) | R


def feistel64(x: torch.Tensor, key: int) -> torch.Tensor:
    """Bijection on 64-bit words (int64 bit patterns)."""
    L = _lsr(x, 32)
    R = x & 0xFFFFFFFF
    for r in range(4):
        kr = _s64(_mix64_int(key * 4 + r + 7 * GOLDEN))
        F = mix64(R ^ kr) & 0xFFFFFFFF
        L, R = R, L ^ F
    return (L << 32) | R


def zipf_u32(n: int, s: float, N: int, seed: int = 0, device="cpu") -> torch.Tensor:
    """Zipf(s) ranks over 1..N mapped to 32-bit keys by a seeded bijection."""
    return feistel32(zipf_ranks(n, s, N, seed, device, stream=6), seed + 11)


def zipf_u64(n: int, s: float, N: int, seed: int = 0, device="cpu") -> torch.Tensor:
    return feistel64(zipf_ranks(n, s, N, seed, device, stream=7), seed + 13)


def mixture_u64(n: int, seed: int = 0, device="cpu") -> torch.Tensor:
    """40% Zipf s=1.2 over 1e8 ranks (bijected to 64 bits), 40% uniform 64-bit,
    20% floor(Exp(1e-9)); the component is chosen by an independent uniform."""
    u = uniform01(seed, 8, n, device)
    z = zipf_u64(n, 1.2, 10 ** 8, seed + 101, device)
    un = uniform_u64(n, seed + 102, device)
    ex = exponential_keys(n, 1e-9, seed + 103, device)
    return torch.where(u < 0.4, z, torch.where(u < 0.8, un, ex))


def segment_sizes(n_seg: int = 4096, median: float = 2.0 ** 14, sigma: float = 1.5,
                  lo: int = 1000, hi: int = 10 ** 7, seed: int = 0, device="cpu") -> torch.Tensor:
    """Log-normal sizes round(median * exp(sigma Z)), Z ~ N(0,1) by Box-Muller, clipped."""
    u1 = uniform01(seed, 9, n_seg, device)
    u2 = uniform01(seed, 10, n_seg, device)
    z = torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos(2.0 * math.pi * u2)
    size = torch.round(median * torch.exp(sigma * z))
    return torch.clamp(size, lo, hi).to(torch.int64)


def segmented_u32(sizes: torch.Tensor, seed: int = 0, device="cpu"):
    """Keys for independent instances: instance i draws uniform 32-bit keys or
    Zipf s in {0.6, 1.0, 1.5} over ranks 1..size_i (bijected), chosen by hash."""
    sizes = sizes.to(device)
    n_seg = sizes.numel()
    offsets = torch.zeros(n_seg + 1, dtype=torch.int64, device=device)
    offsets[1:] = torch.cumsum(sizes, 0)
    total = int(offsets[-1])
    choice = _lsr(rand64(seed, 12, n_seg, device), 1) % 4
    seg_of = torch.repeat_interleave(torch.arange(n_seg, device=device), sizes)
    ch = choice[seg_of]
    keys = uniform_u32(total, seed + 201, device)
    N = sizes[seg_of].to(torch.float64)
    for c, s in ((1, 0.6), (2, 1.0), (3, 1.5)):
        idx = torch.nonzero(ch == c).flatten()
        if idx.numel() == 0:
            continue
        r = zipf_ranks(idx.numel(), s, N[idx], seed + 300 + c, device, stream=13 + c)
        keys[idx] = feistel32(r + seg_of[idx] * 7919, seed + 400 + c) & 0xFFFFFFFF
    return keys, offsets


# ------------------------------------------- the paper's synthetic grid
# Section 6 (Tab. synthetic): Unif-mu (mu distinct keys), Exp-lambda
# (exponential with rate 1e-5 * lambda, rounded to the closest integer),
# Zipf-s (ranks 1..n with P(k) ~ k^-s) and BExp-t (every bit of a key is 0
# with probability 1/t, else 1).  The three standard families are mapped to
# the full key range by a seeded bijection of the key width (the paper maps
# them "to larger ranges ... to test the full range"); BExp keys are used as
# drawn.  Width 32 or 64; int64 bit patterns.
PAPER_GRID = {
    "unif": (10, 10 ** 3, 10 ** 5, 10 ** 7, 10 ** 9),
    "exp": (1, 2, 5, 7, 10),
    "zipf": (0.6, 0.8, 1.0, 1.2, 1.5),
    "bexp": (10, 30, 50, 100, 300),
}

_CHUNK = 1 << 26  # keys generated per pass (bounds temporary memory)


def _biject(x: torch.Tensor, bits: int, key: int) -> torch.Tensor:
    return feistel32(x, key) if bits == 32 else feistel64(x, key)


def paper_bexp(n: int, t: float, bits: int, seed: int = 0, device="cpu", stream: int = 40) -> torch.Tensor:
    """BExp-t: every bit independently 0 with probability 1/t.  A bit is 0
    when its own 32-bit uniform is below floor(2^32 / t) (two bits per 64-bit
    word of the generator)."""
    thr = int((1 << 32) // t)
    out = torch.empty(n, dtype=torch.int64, device=device)
    for c0 in range(0, n, _CHUNK):
        m = min(_CHUNK, n - c0)
        k = torch.zeros(m, dtype=torch.int64, device=device)
        for j in range(bits // 2):
            w = rand64(seed, stream * 64 + j, m, device, start=c0)
            lo = (w & 0xFFFFFFFF) >= thr
            hi = _lsr(w, 32) >= thr
            k |= (lo.to(torch.int64) << (2 * j)) | (hi.to(torch.int64) << (2 * j + 1))
        out[c0:c0 + m] = k
    return out


def paper_keys(family: str, param: float, n: int, bits: int, seed: int = 0, device="cpu") -> torch.Tensor:
    """n keys of one instance of the paper's synthetic grid (see PAPER_GRID)."""
    if bits not in (32, 64):
        raise ValueError("bits must be 32 or 64")
    key = seed * 131 + 17
    if family == "unif":
        mu = int(param)
        out = torch.empty(n, dtype=torch.int64, device=device)
        for c0 in range(0, n, _CHUNK):
            m = min(_CHUNK, n - c0)
            u = uniform01(seed, 30, m, device, start=c0)
            r = torch.clamp(torch.floor(u * mu).to(torch.int64), max=mu - 1)
            out[c0:c0 + m] = _biject(r, bits, key)
        return out
    if family == "exp":
        rate = 1e-5 * float(param)
        out = torch.empty(n, dtype=torch.int64, device=device)
        for c0 in range(0, n, _CHUNK):
            m = min(_CHUNK, n - c0)
            u = uniform01(seed, 31, m, device, start=c0)
            x = torch.round(-torch.log1p(-u) / rate).to(torch.int64)
            out[c0:c0 + m] = _biject(x, bits, key)
        return out
    if family == "zipf":
        r = zipf_ranks(n, float(param), n, seed, device, stream=32)
        return _biject(r, bits, key)
    if family == "bexp":
        return paper_bexp(n, float(param), bits, seed, device)
    raise KeyError(family)


# ------------------------------------------------------- applications
# Synthetic stand-ins for the inputs of the paper's applications (Section
# 6.2; its real graphs and point sets are not available here).


def power_law_graph(n_vertices: int, n_edges: int, s_out: float = 0.8, s_in: float = 1.0, seed: int = 0,
                    device="cpu"):
    """A directed graph in CSR form (offsets int64 [V + 1], targets int64
    [E]) whose out- and in-degrees follow Zipf laws over the vertices (social
    and web graphs: a few vertices with very many edges).  Edge sources are
    Zipf(s_out) ranks and targets Zipf(s_in) ranks, each mapped to vertex ids
    by its own multiplicative bijection of [0, V) (V a power of two)."""
    if n_vertices & (n_vertices - 1):
        raise ValueError("n_vertices must be a power of two")
    mask = n_vertices - 1
    counts = torch.zeros(n_vertices, dtype=torch.int64, device=device)
    for c0 in range(0, n_edges, _CHUNK):
        m = min(_CHUNK, n_edges - c0)
        r = zipf_ranks(m, s_out, n_vertices, seed + c0, device, stream=50)
        u = ((r - 1) * 0x9E3779B1) & mask
        counts += torch.bincount(u, minlength=n_vertices)
    offsets = torch.zeros(n_vertices + 1, dtype=torch.int64, device=device)
    offsets[1:] = torch.cumsum(counts, 0)
    targets = torch.empty(n_edges, dtype=torch.int64, device=device)
    for c0 in range(0, n_edges, _CHUNK):
        m = min(_CHUNK, n_edges - c0)
        r = zipf_ranks(m, s_in, n_vertices, seed + 7 + c0, device, stream=51)
        targets[c0:c0 + m] = ((r - 1) * 0x2545F491) & mask
    return offsets, targets


def varden_points(n: int, dims: int, seed: int = 0, device="cpu", clusters: int = 64) -> torch.Tensor:
    """Points with varying density in [0, 2^(32 // dims))^dims, coords[d][i]
    (int64): a uniform background (10 %) and Gaussian clusters whose
    centres are uniform and whose spreads span four orders of magnitude
    (a stand-in for the varying-density generator the paper uses)."""
    side = 1 << (32 // dims)
    out = torch.empty(dims, n, dtype=torch.int64, device=device)
    cu = uniform01(seed, 60, clusters * dims, device).view(clusters, dims) * side
    sig = side * torch.pow(10.0, -1.0 - 4.0 * uniform01(seed, 61, clusters, device))
    for c0 in range(0, n, _CHUNK):
        m = min(_CHUNK, n - c0)
        pick = (_lsr(rand64(seed, 62, m, device, start=c0), 1) % clusters)
        bg = uniform01(seed, 63, m, device, start=c0) < 0.1
        for d in range(dims):
            u1 = uniform01(seed, 64 + 2 * d, m, device, start=c0)
            u2 = uniform01(seed, 65 + 2 * d, m, device, start=c0)
            g = torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos(2.0 * math.pi * u2)  # Box-Muller
            x = cu[pick, d] + sig[pick] * g
            x = torch.where(bg, u1 * side, x)
            out[d, c0:c0 + m] = torch.clamp(torch.floor(x), 0, side - 1).to(torch.int64)
    return out


# ---------------------------------------------------------------- configs
CONFIGS = {
    # name: (key dtype, has values, default n)
    "uniform_u32_2p20": ("u32", False, 1 << 20),
    "uniform_u32": ("u32", False, 10 ** 9),
    "zipf1_u32": ("u32", False, 10 ** 9),
    "exp_pairs_u64": ("u64", True, 10 ** 9),
    "bexp_pairs_u64": ("u64", True, 10 ** 9),
    "segmented_u32": ("u32", False, None),
    "mixture_u64": ("u64", False, 10 ** 9),
}


def make_config(name: str, n: int | None = None, seed: int = 0, device="cpu", n_seg: int | None = None):
    """Generate one workload.  Returns a dict with 'keys' (int64 bit patterns),
    optionally 'values' (original index) and 'offsets' (segmented)."""
    kt, has_v, n_def = CONFIGS[name]
    n = n_def if n is None else n
    out = {"name": name, "key_type": kt}
    if name == "uniform_u32_2p20" or name == "uniform_u32":
        out["keys"] = uniform_u32(n, seed, device)
    elif name == "zipf1_u32":
        out["keys"] = zipf_u32(n, 1.0, n, seed, device)
    elif name == "exp_pairs_u64":
        out["keys"] = exponential_keys(n, 1e-5, seed, device)
    elif name == "bexp_pairs_u64":
        out["keys"] = bit_exponential_keys(n, 0.1, seed, device)
    elif name == "mixture_u64":
        out["keys"] = mixture_u64(n, seed, device)
    elif name == "segmented_u32":
        ns = 4096 if n_seg is None else n_seg
        sizes = segment_sizes(ns, seed=seed, device=device)
        if n is not None and n < int(sizes.sum()):
            # scaled-down variant for quick tests: same shape, sizes scaled to total ~n
            scale = n / float(sizes.sum())
            sizes = torch.clamp(torch.round(sizes.to(torch.float64) * scale), 1, None).to(torch.int64)
        keys, offsets = segmented_u32(sizes, seed, device)
        out["keys"], out["offsets"] = keys, offsets
    else:
        raise KeyError(name)
    if has_v:
        out["values"] = torch.arange(out["keys"].numel(), dtype=torch.int64, device=device)
    return out
