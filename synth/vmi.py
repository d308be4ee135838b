"""Seeded synthetic TimePix3 velocity-map-imaging workloads.

This module only fabricates inputs.  It draws laser-shot trigger times,
particle hits (Gaussian phosphor spots on the 256 x 256 pixel grid), the pixel
events those spots fire, dark counts and junk packets, and interleaves them
into a stream of 64-bit packets ordered by the time each packet is reported.
It performs none of the processing that the library and the oracle perform
(no decoding, ToA unwrapping, shot assignment, clustering or centroiding).  It
keeps the ground truth of what it generated (absolute arrival times, the shot
and hit each pixel came from) so that tests can pin those steps against it.

Physical model, following the paper's description of the detector:
  * a pixel reports x, y, ToA and ToT only after its signal has dropped below
    threshold, so packets leave the camera in report order, not ToA order
    (Sec. III; Sec. IV, ToA Unwrapping);
  * ToT is counted in 25 ns units and ToA in 1.5625 ns ticks (25/16 ns, i.e.
    256 of the chip's 25/4096 ns units, Sec. IV);
  * trigger (TDC) packets arrive interleaved with pixel packets (Sec. III);
  * dark counts are spread over the whole 1 ms shot period, so only about a
    tenth of them fall inside the 100 us ToF window (Sec. IV, Eliminating
    Background Counts);
  * brighter pixels cross threshold earlier (time walk, Sec. IV, ToT-ToF
    Correlation Correction); here ToA = hit time + 20 ns * (1 - amplitude)
    plus Gaussian jitter.

Packet layout (the paper gives none; this is the project's reading of the
public TPX3 format, kept self-consistent by round-trip tests):
  pixel word  bits 63..60 = 0xB, 59..53 = x >> 1, 52..47 = y >> 2,
              46..44 = ((x & 1) << 2) | (y & 3), 43..30 = coarse ToA (14 b),
              29..20 = ToT (10 b), 19..16 = fine ToA (4 b),
              15..0 = spidr time (16 b);
              arrival tick = (((spidr << 14) | toa) << 4) - ftoa  mod 2^34
  TDC word    bits 63..60 = 0x6, 59..56 = subtype (0xF = TDC1 rising edge),
              55..44 = trigger counter (12 b), 43..9 = timestamp in
              3.125 ns units (35 b), 8..5 = fine (4 b, unused);
              trigger tick = 2 * timestamp  mod 2^36
"""
from __future__ import annotations

import dataclasses
import math
import multiprocessing
import os

import numpy as np

TICK_NS = 1.5625                  # 25/16 ns
TOT_TICKS = 16                    # one 25 ns ToT count in ToA ticks
SHOT_PERIOD_TICKS = 640_000       # 1 kHz laser
PIX_WRAP_TICKS = 1 << 34          # 2^42 units of 25/4096 ns = 26.84 s
TDC_WRAP_TICKS = 1 << 36          # 2^44 units of 25/4096 ns = 107.37 s
GRID = 256
TRIG_SUBTYPE = 0xF                # TDC1 rising edge
FALL_SUBTYPE = 0xA                # TDC1 falling edge (not a trigger)
HDR_PIXEL = 0xB
HDR_TDC = 0x6
HDR_JUNK = 0x4                    # e.g. global-time / control words
AMP_KEEP = 0.05                   # pixels kept where amplitude >= 5 % of peak
MERGE_NS = 1000.0                 # same-pixel contributions closer than this
                                  # fire one event (pixel still over threshold)
SHOTS_PER_BATCH = 2000

KIND_PIXEL, KIND_TRIGGER, KIND_OTHER = 0, 1, 2


# --------------------------------------------------------------------------
# packet encoding (the generator's own copy of the layout above)
# --------------------------------------------------------------------------
def encode_pixels(x, y, tot, t_abs):
    """Pack pixel events into 64-bit words; t_abs in ticks (any epoch)."""
    x = np.asarray(x, dtype=np.uint64)
    y = np.asarray(y, dtype=np.uint64)
    tot = np.asarray(tot, dtype=np.uint64)
    raw = np.asarray(t_abs, dtype=np.int64) % PIX_WRAP_TICKS
    raw = raw.astype(np.uint64)
    coarse = ((raw + np.uint64(15)) >> np.uint64(4))          # ceil(raw / 16)
    ftoa = (coarse << np.uint64(4)) - raw                      # 0..15
    coarse = coarse & np.uint64((1 << 30) - 1)
    spidr = coarse >> np.uint64(14)
    toa = coarse & np.uint64(0x3FFF)
    pix = ((x & np.uint64(1)) << np.uint64(2)) | (y & np.uint64(3))
    w = (np.uint64(HDR_PIXEL) << np.uint64(60)) \
        | ((x >> np.uint64(1)) << np.uint64(53)) \
        | ((y >> np.uint64(2)) << np.uint64(47)) \
        | (pix << np.uint64(44)) \
        | (toa << np.uint64(30)) \
        | ((tot & np.uint64(0x3FF)) << np.uint64(20)) \
        | (ftoa << np.uint64(16)) \
        | spidr
    return w.astype(np.uint64)


def encode_tdc(t_abs, counter, subtype=TRIG_SUBTYPE, fine=0):
    """Pack TDC words; t_abs in ticks, must be even (3.125 ns resolution)."""
    t = np.asarray(t_abs, dtype=np.int64)
    if np.any(t % 2):
        raise ValueError("TDC times must be even ticks")
    ts = ((t % TDC_WRAP_TICKS) // 2).astype(np.uint64)
    counter = np.asarray(counter, dtype=np.uint64) & np.uint64(0xFFF)
    sub = np.broadcast_to(np.asarray(subtype, dtype=np.uint64), ts.shape)
    fine = np.broadcast_to(np.asarray(fine, dtype=np.uint64), ts.shape)
    w = (np.uint64(HDR_TDC) << np.uint64(60)) | (sub << np.uint64(56)) \
        | (counter << np.uint64(44)) | (ts << np.uint64(9)) \
        | ((fine & np.uint64(0xF)) << np.uint64(5))
    return w.astype(np.uint64)


def encode_junk(rng, n):
    payload = rng.integers(0, 1 << 60, size=n, dtype=np.int64).astype(np.uint64)
    return ((np.uint64(HDR_JUNK) << np.uint64(60)) | payload).astype(np.uint64)


# --------------------------------------------------------------------------
# workload specifications
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class HitKind:
    weight: float
    sigma: tuple          # (lo, hi) px, uniform
    tot_scale: tuple      # (lo, hi): ToT = rint(scale * amplitude), uniform


@dataclasses.dataclass(frozen=True)
class Spec:
    name: str
    seed: int
    n_shots: int
    t0_ticks: int                         # absolute time of the first trigger
    hit_mix: tuple                        # ((weight, poisson_mean), ...)
    kinds: tuple                          # HitKind, ...
    pair_frac: float = 0.0                # hits planted as a close partner
    pair_sep_px: tuple = (1.0, 4.0)
    pair_dt_ns: tuple = (0.0, 50.0)
    hit_window_ns: float = 10_000.0       # hit times U[0, 10 us) after trigger
    walk_ns: float = 20.0                 # ToA += walk_ns * (1 - amplitude)
    jitter_ns: float = 1.5
    noise_frac: float = 0.01              # dark counts per signal pixel
    n_pre_trigger: int = 7                # dark counts before the first trigger
    delay_max_ticks: int = 6400           # readout delay U[0, 10 us)
    fall_edges: bool = True               # a falling-edge TDC after each trigger
    junk_per_shot: float = 0.05           # non-pixel, non-TDC words


ELECTRON_08 = HitKind(1.0, (0.8, 0.8), (400.0, 400.0))

SPECS = {
    # small plain-method case: 1,000 shots, Poisson(10) hits, sigma 0.8 px
    "c1": Spec("c1", 1001, 1000, SHOT_PERIOD_TICKS, ((1.0, 10.0),),
               (ELECTRON_08,)),
    # plain method at scale: 100,000 shots, Poisson(30), sigma U(0.6, 1.5),
    # 10 % close pairs; starts 60 s into the acquisition so that three pixel
    # wraps and one trigger wrap (coinciding at 107.37 s) fall inside the run
    "c2": Spec("c2", 1002, 100_000, 38_400_000_000, ((1.0, 30.0),),
               (HitKind(1.0, (0.6, 1.5), (400.0, 400.0)),), pair_frac=0.10),
    # uneven shots: mixture of Poisson(5), Poisson(40), Poisson(200);
    # 60 % electron-like (sigma 0.5), 40 % ion-like (sigma 1.5-2.5,
    # ToT scale up to 1023)
    "c3": Spec("c3", 1003, 200_000, 6_400_000_000,
               ((0.70, 5.0), (0.25, 40.0), (0.05, 200.0)),
               (HitKind(0.6, (0.5, 0.5), (400.0, 400.0)),
                HitKind(0.4, (1.5, 2.5), (400.0, 1023.0)))),
    # streaming: 1 kHz, Poisson(100) hits/shot, sigma 0.8; starts 2 s before
    # the 26.84 s pixel wrap so that a wrap lands inside the replay
    "c5": Spec("c5", 1005, 5_000, PIX_WRAP_TICKS - 1_280_000_000,
               ((1.0, 100.0),), (ELECTRON_08,)),
}


@dataclasses.dataclass
class Workload:
    spec: Spec
    packets: np.ndarray                   # uint64, stream order
    pix_epoch0: int
    tdc_epoch0: int
    trig_ticks: np.ndarray                # int64, absolute, trigger k
    trig_pos: np.ndarray | None = None    # int64, stream index of trigger k's word
    # per-packet truth (stream order); None when generated without truth
    kind: np.ndarray | None = None        # KIND_*
    t_abs: np.ndarray | None = None       # int64 absolute ticks (pixels, TDCs)
    x: np.ndarray | None = None
    y: np.ndarray | None = None
    tot: np.ndarray | None = None
    shot: np.ndarray | None = None        # int64 originating shot, -1 before T[0]
    tof: np.ndarray | None = None         # int64 ticks after that shot's trigger
    hit: np.ndarray | None = None         # int64 originating hit, -1 dark count
    # per-hit truth
    hit_shot: np.ndarray | None = None
    hit_x: np.ndarray | None = None       # true sub-pixel centre
    hit_y: np.ndarray | None = None
    hit_t_ns: np.ndarray | None = None    # true hit time after the trigger
    hit_sigma: np.ndarray | None = None

    @property
    def n_packets(self):
        return int(self.packets.size)

    def kept_mask(self, tof_max_ticks=64_000):
        """Pixels that a correct decode keeps: after a trigger and within the
        ToF window of the shot they were generated in."""
        return (self.kind == KIND_PIXEL) & (self.shot >= 0) \
            & (self.tof <= tof_max_ticks)


def _draw_hits_per_shot(rng, spec, n):
    w = np.array([m[0] for m in spec.hit_mix])
    lam = np.array([m[1] for m in spec.hit_mix])
    comp = rng.choice(len(w), size=n, p=w / w.sum())
    return rng.poisson(lam[comp]).astype(np.int64)


def _draw_hits(rng, spec, shot_lo, shot_hi):
    nh = _draw_hits_per_shot(rng, spec, shot_hi - shot_lo)
    shot = np.repeat(np.arange(shot_lo, shot_hi, dtype=np.int64), nh)
    H = shot.size
    kw = np.array([k.weight for k in spec.kinds])
    kind = rng.choice(len(kw), size=H, p=kw / kw.sum())
    s_lo = np.array([k.sigma[0] for k in spec.kinds])[kind]
    s_hi = np.array([k.sigma[1] for k in spec.kinds])[kind]
    c_lo = np.array([k.tot_scale[0] for k in spec.kinds])[kind]
    c_hi = np.array([k.tot_scale[1] for k in spec.kinds])[kind]
    sigma = s_lo + (s_hi - s_lo) * rng.random(H)
    scale = c_lo + (c_hi - c_lo) * rng.random(H)
    cx = rng.random(H) * GRID
    cy = rng.random(H) * GRID
    t_ns = rng.random(H) * spec.hit_window_ns
    if spec.pair_frac > 0 and H > 1:
        partner = rng.random(H) < spec.pair_frac
        partner[0] = False
        partner[1:] &= shot[1:] == shot[:-1]
        partner[1:] &= ~partner[:-1]          # no chains of partners
        idx = np.nonzero(partner)[0]
        sep = spec.pair_sep_px[0] + (spec.pair_sep_px[1] - spec.pair_sep_px[0]) \
            * rng.random(idx.size)
        phi = rng.random(idx.size) * 2 * math.pi
        dt = spec.pair_dt_ns[0] + (spec.pair_dt_ns[1] - spec.pair_dt_ns[0]) \
            * rng.random(idx.size)
        cx[idx] = np.clip(cx[idx - 1] + sep * np.cos(phi), 0, GRID - 1e-9)
        cy[idx] = np.clip(cy[idx - 1] + sep * np.sin(phi), 0, GRID - 1e-9)
        t_ns[idx] = np.minimum(t_ns[idx - 1] + dt, spec.hit_window_ns)
    return shot, cx, cy, t_ns, sigma, scale


def _expand_spots(cx, cy, sigma, scale):
    """Pixels of each Gaussian spot with amplitude >= AMP_KEEP (pixel centres
    at integer coordinates).  Returns hit index, px, py, amplitude, ToT part."""
    r = sigma * math.sqrt(2.0 * math.log(1.0 / AMP_KEEP))
    R = np.ceil(r).astype(np.int64)
    outs = []
    for Rv in np.unique(R):
        m = np.nonzero(R == Rv)[0]
        offs = np.arange(-Rv, Rv + 2, dtype=np.int64)
        ox, oy = np.meshgrid(offs, offs, indexing="ij")
        ox = ox.ravel()
        oy = oy.ravel()
        bx = np.floor(cx[m]).astype(np.int64)
        by = np.floor(cy[m]).astype(np.int64)
        px = bx[:, None] + ox[None, :]
        py = by[:, None] + oy[None, :]
        d2 = (px - cx[m, None]) ** 2 + (py - cy[m, None]) ** 2
        amp = np.exp(-d2 / (2.0 * sigma[m, None] ** 2))
        keep = (amp >= AMP_KEEP) & (px >= 0) & (px < GRID) & (py >= 0) & (py < GRID)
        hi = np.broadcast_to(m[:, None], px.shape)[keep]
        outs.append((hi, px[keep], py[keep], amp[keep]))
    hi = np.concatenate([o[0] for o in outs])
    px = np.concatenate([o[1] for o in outs])
    py = np.concatenate([o[2] for o in outs])
    amp = np.concatenate([o[3] for o in outs])
    return hi, px, py, amp, amp * scale[hi]


def _batch(rng, spec, shot_lo, shot_hi, trig, hit_base):
    """Events, triggers and junk of shots [shot_lo, shot_hi)."""
    hshot, cx, cy, t_ns, sigma, scale = _draw_hits(rng, spec, shot_lo, shot_hi)
    hi, px, py, amp, totc = _expand_spots(cx, cy, sigma, scale)
    # one event per (shot, pixel) and per merge window; ToT from the summed
    # light, ToA from the earliest contributing hit
    key = ((hshot[hi] - shot_lo) << 16) | (py << 8) | px
    th = t_ns[hi]
    order = np.lexsort((th, key))
    key, th, hi, amp, totc = key[order], th[order], hi[order], amp[order], totc[order]
    new = np.ones(key.size, dtype=bool)
    if key.size:
        new[1:] = (key[1:] != key[:-1]) | (th[1:] - th[:-1] > MERGE_NS)
    eid = np.cumsum(new) - 1
    first = np.nonzero(new)[0]
    ne = first.size
    amp_sum = np.bincount(eid, weights=amp, minlength=ne)
    tot_sum = np.bincount(eid, weights=totc, minlength=ne)
    e_hit = hi[first]
    e_t = th[first]
    e_key = key[first]
    e_x = (e_key & 0xFF).astype(np.int64)
    e_y = ((e_key >> 8) & 0xFF).astype(np.int64)
    e_shot = hshot[e_hit]
    e_tot = np.clip(np.rint(tot_sum), 1, 1023).astype(np.int64)
    walk = spec.walk_ns * (1.0 - np.minimum(amp_sum, 1.0))
    tof_ns = e_t + walk + rng.normal(0.0, spec.jitter_ns, ne)
    e_tof = np.maximum(0, np.rint(tof_ns / TICK_NS)).astype(np.int64)
    e_tabs = trig[e_shot] + e_tof

    # dark counts: uniform over the whole shot period of a random shot
    n_noise = int(round(spec.noise_frac * ne))
    n_shot = rng.integers(shot_lo, shot_hi, n_noise)
    n_off = rng.integers(0, SHOT_PERIOD_TICKS, n_noise)
    n_x = rng.integers(0, GRID, n_noise)
    n_y = rng.integers(0, GRID, n_noise)
    n_tot = rng.integers(1, 401, n_noise)
    if shot_lo == 0 and spec.n_pre_trigger:
        k = spec.n_pre_trigger
        n_shot = np.concatenate([np.full(k, -1), n_shot])
        n_off = np.concatenate([-rng.integers(1, 100_000, k), n_off])
        n_x = np.concatenate([rng.integers(0, GRID, k), n_x])
        n_y = np.concatenate([rng.integers(0, GRID, k), n_y])
        n_tot = np.concatenate([rng.integers(1, 401, k), n_tot])
    n_tabs = np.where(n_shot >= 0, trig[np.maximum(n_shot, 0)] + n_off,
                      trig[0] + n_off)

    x = np.concatenate([e_x, n_x])
    y = np.concatenate([e_y, n_y])
    tot = np.concatenate([e_tot, n_tot])
    tabs = np.concatenate([e_tabs, n_tabs])
    shot = np.concatenate([e_shot, n_shot])
    tof = np.concatenate([e_tof, np.where(n_shot >= 0, n_off, -1)])
    hit = np.concatenate([e_hit + hit_base, np.full(n_shot.size, -1)])
    rt = tabs + TOT_TICKS * tot + rng.integers(0, spec.delay_max_ticks, tabs.size)
    kind = np.full(tabs.size, KIND_PIXEL)

    # triggers (and their falling edges, which are not triggers)
    ks = np.arange(shot_lo, shot_hi, dtype=np.int64)
    t_trig = trig[ks]
    parts = dict(kind=[kind, np.full(ks.size, KIND_TRIGGER)],
                 x=[x, np.zeros(ks.size, np.int64)], y=[y, np.zeros(ks.size, np.int64)],
                 tot=[tot, np.zeros(ks.size, np.int64)], t_abs=[tabs, t_trig],
                 shot=[shot, ks], tof=[tof, np.zeros(ks.size, np.int64)],
                 hit=[hit, np.full(ks.size, -1)], rt=[rt, t_trig],
                 sub=[np.zeros(tabs.size, np.int64), np.full(ks.size, TRIG_SUBTYPE)])
    if spec.fall_edges:
        parts["kind"].append(np.full(ks.size, KIND_OTHER))
        for f in ("x", "y", "tot", "tof"):
            parts[f].append(np.zeros(ks.size, np.int64))
        parts["t_abs"].append(t_trig + 1280)
        parts["shot"].append(ks)
        parts["hit"].append(np.full(ks.size, -1))
        parts["rt"].append(t_trig + 1280)
        parts["sub"].append(np.full(ks.size, FALL_SUBTYPE))
    n_junk = rng.poisson(spec.junk_per_shot * ks.size)
    if n_junk:
        jt = trig[shot_lo] + rng.integers(0, SHOT_PERIOD_TICKS * ks.size, n_junk)
        parts["kind"].append(np.full(n_junk, KIND_OTHER))
        for f in ("x", "y", "tot", "tof"):
            parts[f].append(np.zeros(n_junk, np.int64))
        parts["t_abs"].append(jt)
        parts["shot"].append(np.full(n_junk, -1))
        parts["hit"].append(np.full(n_junk, -1))
        parts["rt"].append(jt)
        parts["sub"].append(np.full(n_junk, -1))
    out = {k: np.concatenate(v) for k, v in parts.items()}
    hits = dict(hit_shot=hshot, hit_x=cx, hit_y=cy, hit_t_ns=t_ns, hit_sigma=sigma)
    return out, hits


def make_config(name, seed=None, n_shots=None, with_truth=True, workers=None):
    """Generate one of the workloads 'c1', 'c2', 'c3', 'c5'.

    ``n_shots`` shrinks a workload to fewer shots with the same distributions
    (used for parity tests that the oracle finishes in seconds)."""
    spec = SPECS[name]
    if seed is not None or n_shots is not None:
        spec = dataclasses.replace(spec, seed=spec.seed if seed is None else seed,
                                   n_shots=spec.n_shots if n_shots is None else n_shots)
    return generate(spec, with_truth=with_truth, workers=workers)


def _batch_job(args):
    spec, seed_seq, lo, hi, trig = args
    rng = np.random.Generator(np.random.PCG64(seed_seq))
    return _batch(rng, spec, lo, hi, trig, 0)


def generate(spec, with_truth=True, workers=None):
    """Build the packet stream of ``spec``.  Shots are drawn in batches of
    SHOTS_PER_BATCH, each from its own child of the seed's SeedSequence, so
    the result does not depend on ``workers`` (parallel batch drawing)."""
    S = spec.n_shots
    trig = spec.t0_ticks + SHOT_PERIOD_TICKS * np.arange(S + 1, dtype=np.int64)
    bounds = [(lo, min(S, lo + SHOTS_PER_BATCH)) for lo in range(0, S, SHOTS_PER_BATCH)]
    seqs = np.random.SeedSequence(spec.seed).spawn(len(bounds) + 1)
    jobs = [(spec, seqs[i], lo, hi, trig) for i, (lo, hi) in enumerate(bounds)]
    if workers is None:
        workers = int(os.environ.get("TPX_SYNTH_WORKERS", "1"))
    if workers > 1 and len(jobs) > 2:
        ctx = multiprocessing.get_context("fork")
        with ctx.Pool(min(workers, len(jobs))) as pool:
            results = pool.imap(_batch_job, jobs)
            return _assemble(spec, trig, bounds, results, seqs[-1], with_truth)
    return _assemble(spec, trig, bounds, map(_batch_job, jobs), seqs[-1], with_truth)


def _assemble(spec, trig, bounds, results, junk_seq, with_truth):
    S = spec.n_shots
    jrng = np.random.Generator(np.random.PCG64(junk_seq))
    fields = ("kind", "x", "y", "tot", "t_abs", "shot", "tof", "hit", "sub")
    chunks = {f: [] for f in fields}
    chunks["pk"] = []
    hit_chunks = {f: [] for f in ("hit_shot", "hit_x", "hit_y", "hit_t_ns", "hit_sigma")}
    carry = None
    hit_base = 0
    n_out = 0
    trig_pos = []
    for (lo, hi), (b, hits) in zip(bounds, results):
        b["hit"] = np.where(b["hit"] >= 0, b["hit"] + hit_base, -1)
        hit_base += hits["hit_shot"].size
        if with_truth:
            for f in hit_chunks:
                hit_chunks[f].append(hits[f])
        if carry is not None:
            b = {k: np.concatenate([carry[k], b[k]]) for k in b}
        # stream order: report time, then triggers before pixels before others
        cls = np.where(b["kind"] == KIND_TRIGGER, 0, np.where(b["kind"] == KIND_PIXEL, 1, 2))
        order = np.argsort(b["rt"] * 4 + cls, kind="stable")
        b = {k: v[order] for k, v in b.items()}
        if hi < S:
            cut = np.searchsorted(b["rt"], trig[hi], side="left")
            carry = {k: v[cut:] for k, v in b.items()}
            b = {k: v[:cut] for k, v in b.items()}
        else:
            carry = None
        pk = np.empty(b["kind"].size, dtype=np.uint64)
        m = b["kind"] == KIND_PIXEL
        pk[m] = encode_pixels(b["x"][m], b["y"][m], b["tot"][m], b["t_abs"][m])
        m = b["sub"] == TRIG_SUBTYPE
        pk[m] = encode_tdc(b["t_abs"][m], b["shot"][m], TRIG_SUBTYPE)
        trig_pos.append(n_out + np.nonzero(m)[0])
        n_out += pk.size
        m = b["sub"] == FALL_SUBTYPE
        pk[m] = encode_tdc(b["t_abs"][m], b["shot"][m], FALL_SUBTYPE)
        m = (b["kind"] == KIND_OTHER) & (b["sub"] < 0)
        if m.any():
            pk[m] = encode_junk(jrng, int(m.sum()))
        chunks["pk"].append(pk)
        if with_truth:
            for f in fields:
                chunks[f].append(b[f])
        else:
            # keep only what the initial epochs need
            for f in ("kind", "t_abs"):
                if not chunks[f]:
                    chunks[f].append(b[f])
    packets = np.concatenate(chunks["pk"])
    kind0 = np.concatenate(chunks["kind"])
    t0 = np.concatenate(chunks["t_abs"])
    first_pix = np.nonzero(kind0 == KIND_PIXEL)[0]
    first_trg = np.nonzero(kind0 == KIND_TRIGGER)[0]
    pix_epoch0 = int(t0[first_pix[0]] // PIX_WRAP_TICKS) if first_pix.size else 0
    tdc_epoch0 = int(t0[first_trg[0]] // TDC_WRAP_TICKS) if first_trg.size else 0
    wl = Workload(spec=spec, packets=packets, pix_epoch0=pix_epoch0,
                  tdc_epoch0=tdc_epoch0, trig_ticks=trig[:S].copy(),
                  trig_pos=np.concatenate(trig_pos).astype(np.int64) if trig_pos else None)
    if with_truth:
        for f in ("kind", "x", "y", "tot", "t_abs", "shot", "tof", "hit"):
            setattr(wl, f, np.concatenate(chunks[f]))
        for f in hit_chunks:
            setattr(wl, f, np.concatenate(hit_chunks[f]))
    return wl


# --------------------------------------------------------------------------
# small event sets for clustering tests (event mode)
# --------------------------------------------------------------------------
def tiny_events(rng, n, grid=6, t_span=400, n_shots=2, sort_by_shot=True,
                repeat_frac=0.2, tot_zero_frac=0.05):
    """Random pixel events on a small grid and short time span, so that
    neighbourhoods, time chains and same-address repeats are frequent.
    Returns dict of x, y, tot (uint16), shot (uint32), toa (uint64) and the
    trigger times (uint64) that the shots refer to."""
    trig = (1_000_000 + SHOT_PERIOD_TICKS * np.arange(max(n_shots, 1))).astype(np.int64)
    shot = rng.integers(0, max(n_shots, 1), n)
    if sort_by_shot:
        shot = np.sort(shot)
    x = rng.integers(0, grid, n)
    y = rng.integers(0, grid, n)
    if n > 1:
        rep = np.nonzero(rng.random(n) < repeat_frac)[0]
        src = rng.integers(0, n, rep.size)
        x[rep] = x[src]
        y[rep] = y[src]
    off = rng.integers(0, t_span + 1, n)
    tot = rng.integers(1, 1024, n)
    tot[rng.random(n) < tot_zero_frac] = 0
    toa = trig[shot] + off
    return dict(x=x.astype(np.uint16), y=y.astype(np.uint16), tot=tot.astype(np.uint16),
                shot=shot.astype(np.uint32), toa=toa.astype(np.uint64),
                trig=trig.astype(np.uint64))
