"""Long permanents as resumable segments of the Gray-code range.

A sweep at n = 45..52 runs for minutes to hours on one device.  The parallel
listings of the paper's Supplementary (Algorithms S1 and S2) already cut the
term index k into contiguous ranges whose partial sums are reduced at the
end; this module applies the same cut in time as well as across devices:

* the 2^(n-1) (BB/FG) or 2^n (Ryser) terms are split into S segments of
  2^s terms, segment i covering [i 2^s, (i+1) 2^s), each evaluated by
  ph_perm_partial into one double-double partial;
* after every segment the partial (as exact hex floats), its duration and the
  index of the next segment are written to a checkpoint file, atomically
  (temporary file, fsync, rename);
* a run that stops (crash, kill, time limit) is restarted from the
  checkpoint: it checks that the file belongs to the same matrix, formula,
  accumulation, chunk length, segment length, shard and device, and goes on at
  the first missing segment;
* the total is ph_perm_combine of all partials in segment order, so a run
  interrupted any number of times gives the same bits as one that was not;
* a segment that takes more than `slow_factor` times the median of the
  segments before it is recorded as slow (the stand-in for the slow-node
  detection the paper's runs lacked).

Sharding: shard g of G takes the contiguous segments [g S / G, (g+1) S / G),
as device g of G would; `combine_shards` joins the shards' partials in shard
order.  On one device the shards simply run one after another.

Host logic only: the partial sums run in ph_perm_partial and the final
reduction in ph_perm_combine.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
import time
from typing import Callable, Sequence

FORMAT = "permhip-segments-1"

Executor = Callable[[int, int], Sequence[float]]


def _hex4(v: Sequence[float]) -> list:
    return [float(x).hex() for x in v]


def _unhex4(v: Sequence[str]) -> list:
    return [float.fromhex(x) for x in v]


def gpu_executor(a, algo="glynn", accum="dd", chunk_log2: int = 0, waves: int = 0) -> Executor:
    """ph_perm_partial on a's device; each call waits for its segment and
    returns the 4 doubles on the host."""
    from . import permhip

    def run(k_begin: int, k_end: int):
        out = permhip.perm_partial(a, k_begin, k_end, algo, accum, chunk_log2, waves)
        return [float(x) for x in out.cpu().tolist()]

    return run


def gpu_combiner(device, n: int, algo="glynn", accum="dd") -> Callable[[list], complex]:
    """ph_perm_combine of host partials (uploaded in segment order)."""
    import torch

    from . import permhip

    def combine(partials: list) -> complex:
        t = torch.tensor(partials, dtype=torch.float64, device=device).reshape(-1, 4)
        return complex(permhip.perm_combine(t, n, algo, accum).cpu())

    return combine


def device_tag(device) -> str:
    """Name and compute-unit count: the partials' bits depend on the launch
    grid, which follows from these."""
    import torch

    p = torch.cuda.get_device_properties(device)
    return f"{p.name}/{p.multi_processor_count}cu"


class SegmentedPermanent:
    """One permanent (or one shard of it) as checkpointed segments.

    n, algo, accum, chunk_log2: as ph_perm_partial (chunk_log2 is the
    resolved chunk length, perm_chunk_log2(n, ...)).  segment_log2: log2 of
    the terms per segment, at least chunk_log2 and at most the term count.
    fingerprint: bytes identifying the matrix (e.g. its raw bytes).
    executor(k_begin, k_end) -> 4 floats; combiner(list of partials) -> Per.
    clock: seconds, for the segment durations.
    """

    def __init__(self, n: int, algo: str, accum: str, chunk_log2: int, segment_log2: int, fingerprint: bytes,
                 executor: Executor, combiner: Callable[[list], complex], checkpoint: str | None = None,
                 shard: tuple = (0, 1), device: str = "", slow_factor: float = 3.0,
                 clock: Callable[[], float] = time.perf_counter):
        nb = n - 1 if algo == "glynn" else n
        if not 0 <= chunk_log2 <= segment_log2 <= nb:
            raise ValueError(f"need chunk_log2 {chunk_log2} <= segment_log2 {segment_log2} <= {nb}")
        g, G = shard
        if not (G >= 1 and 0 <= g < G):
            raise ValueError(f"bad shard {shard}")
        self.n, self.algo, self.accum = n, algo, accum
        self.segment_log2 = segment_log2
        self.nseg_total = 1 << (nb - segment_log2)
        self.seg_begin = self.nseg_total * g // G
        self.seg_end = self.nseg_total * (g + 1) // G
        self.executor, self.combiner = executor, combiner
        self.checkpoint = checkpoint
        self.slow_factor = slow_factor
        self.clock = clock
        self.key = {
            "sha256": hashlib.sha256(fingerprint).hexdigest(), "n": n, "algo": algo, "accum": accum,
            "chunk_log2": chunk_log2, "segment_log2": segment_log2, "shard": [g, G], "device": device,
        }
        self.partials: list = []
        self.seconds: list = []
        self.slow: list = []
        if checkpoint and os.path.exists(checkpoint):
            self._load()

    # -------------------------------------------------------------- state
    @property
    def next_segment(self) -> int:
        return self.seg_begin + len(self.partials)

    @property
    def done(self) -> bool:
        return self.next_segment >= self.seg_end

    def _load(self):
        with open(self.checkpoint) as f:
            st = json.load(f)
        if st.get("format") != FORMAT:
            raise ValueError(f"{self.checkpoint}: not a segment checkpoint")
        if st["key"] != self.key:
            diff = {k: (st["key"].get(k), v) for k, v in self.key.items() if st["key"].get(k) != v}
            raise ValueError(f"{self.checkpoint} belongs to another run: {diff}")
        if st["next_segment"] != self.seg_begin + len(st["partials"]):
            raise ValueError(f"{self.checkpoint}: next_segment does not match the stored partials")
        self.partials = [_unhex4(p) for p in st["partials"]]
        self.seconds = list(st["seconds"])
        self.slow = list(st["slow"])

    def _save(self):
        if not self.checkpoint:
            return
        st = {"format": FORMAT, "key": self.key, "next_segment": self.next_segment,
              "partials": [_hex4(p) for p in self.partials], "seconds": self.seconds, "slow": self.slow}
        tmp = self.checkpoint + ".tmp"
        with open(tmp, "w") as f:
            json.dump(st, f)
            f.flush()
            os.fsync(f.fileno())
        os.replace(tmp, self.checkpoint)

    # ---------------------------------------------------------------- run
    def run(self, max_segments: int | None = None, progress: Callable[[str], None] | None = None) -> bool:
        """Evaluate up to max_segments further segments (all if None),
        checkpointing after each; returns whether the shard is complete."""
        todo = self.seg_end - self.next_segment
        if max_segments is not None:
            todo = min(todo, max_segments)
        L = 1 << self.segment_log2
        for _ in range(todo):
            i = self.next_segment
            t0 = self.clock()
            part = [float(x) for x in self.executor(i * L, (i + 1) * L)]
            dt = self.clock() - t0
            if len(part) != 4:
                raise ValueError("an executor returns 4 floats")
            if len(self.seconds) >= 3 and dt > self.slow_factor * statistics.median(self.seconds):
                self.slow.append(i)
            self.partials.append(part)
            self.seconds.append(dt)
            self._save()
            if progress:
                progress(f"segment {i + 1}/{self.nseg_total} in {dt:.2f} s")
        return self.done

    def total(self) -> complex:
        if not self.done:
            raise RuntimeError(f"segments {self.next_segment}..{self.seg_end - 1} are missing")
        if self.key["shard"] != [0, 1]:
            raise RuntimeError("a shard has no total of its own: use combine_shards")
        return self.combiner(self.partials)


def combine_shards(shards: Sequence[SegmentedPermanent]) -> complex:
    """Per from complete shards 0..G-1 of one permanent, partials in segment
    order."""
    if not shards:
        raise ValueError("no shards")
    G = shards[0].key["shard"][1]
    if sorted(s.key["shard"][0] for s in shards) != list(range(G)) or any(s.key["shard"][1] != G for s in shards):
        raise ValueError("need shards 0..G-1 of one split")
    base = {k: v for k, v in shards[0].key.items() if k != "shard"}
    for s in shards:
        if {k: v for k, v in s.key.items() if k != "shard"} != base:
            raise ValueError("shards of different runs")
        if not s.done:
            raise RuntimeError(f"shard {s.key['shard']} is incomplete")
    parts = []
    for s in sorted(shards, key=lambda s: s.key["shard"][0]):
        parts.extend(s.partials)
    return shards[0].combiner(parts)


def segmented_perm(a, segment_log2: int, checkpoint: str | None = None, algo="glynn", accum="dd",
                   chunk_log2: int = 0, shard: tuple = (0, 1), max_segments: int | None = None,
                   progress: Callable[[str], None] | None = None) -> SegmentedPermanent:
    """Run (or resume) Per(a) of a complex128 CUDA matrix as checkpointed
    segments of 2^segment_log2 terms on a's device; returns the runner
    (`.total()` once `.done`)."""
    from . import permhip

    n = a.shape[0]
    c = permhip.perm_chunk_log2(n, algo, accum, chunk_log2)
    fp = a.detach().contiguous().cpu().numpy().tobytes()
    r = SegmentedPermanent(n, algo, accum, c, segment_log2, fp, gpu_executor(a, algo, accum, c),
                           gpu_combiner(a.device, n, algo, accum), checkpoint, shard, device_tag(a.device))
    r.run(max_segments, progress)
    return r


def main(argv=None) -> int:
    """Command line: Per of a matrix saved with numpy (.npy, complex, n x n)
    as checkpointed segments on the current GPU; prints progress and a JSON
    line.  Run it again with the same arguments to resume."""
    import argparse

    import numpy as np
    import torch

    ap = argparse.ArgumentParser(prog="python -m paper_1606_05836_amd.segments")
    ap.add_argument("matrix", help=".npy file with an n x n complex matrix")
    ap.add_argument("--segment-log2", type=int, default=40, help="log2 of the terms per segment (clamped)")
    ap.add_argument("--checkpoint", default="", help="checkpoint file (resumed when it exists)")
    ap.add_argument("--algo", default="glynn", choices=("glynn", "ryser"))
    ap.add_argument("--accum", default="dd", choices=("dd", "plain"))
    ap.add_argument("--shard", default="0/1", help="g/G: run shard g of G (the total needs all G)")
    ap.add_argument("--max-segments", type=int, default=None, help="stop after this many new segments")
    args = ap.parse_args(argv)
    a_np = np.load(args.matrix, allow_pickle=False).astype(np.complex128)
    if a_np.ndim != 2 or a_np.shape[0] != a_np.shape[1] or a_np.shape[0] < 1:
        raise SystemExit("the matrix must be n x n with n >= 1")
    g, G = (int(x) for x in args.shard.split("/"))
    from . import permhip

    n = a_np.shape[0]
    c = permhip.perm_chunk_log2(n, args.algo, args.accum)
    nb = n - 1 if args.algo == "glynn" else n
    seg = max(c, min(args.segment_log2, nb))
    a = torch.from_numpy(a_np).to("cuda")
    r = segmented_perm(a, seg, args.checkpoint or None, args.algo, args.accum, shard=(g, G),
                       max_segments=args.max_segments, progress=lambda m: print(m, flush=True))
    out = {"n": n, "algo": args.algo, "accum": args.accum, "segment_log2": seg, "shard": [g, G],
           "done": r.done, "next_segment": r.next_segment, "segments": [r.seg_begin, r.seg_end],
           "seconds": sum(r.seconds), "slow_segments": r.slow}
    if r.done and G == 1:
        p = r.total()
        out["permanent"] = [p.real, p.imag]
    elif r.done:
        out["partials"] = [[x.hex() for x in q] for q in r.partials]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
