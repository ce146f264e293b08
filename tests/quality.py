"""Track-quality tools against generator truth (test helpers).

A *segment* is the part of one particle's path inside one sector on one leg
(outgoing, or the returning half-turn of a looper).  A segment is
reconstructable with >= 30 clusters.  A track matches the segment that owns
>= 90% of its hits; a track matching none is a fake; further tracks matching
an already found segment are clones.
"""
from __future__ import annotations

import numpy as np


def segment_keys(ev) -> np.ndarray:
    """int64 key per cluster: (pid, sector, leg) packed; -1 for noise."""
    key = (ev.pid.astype(np.int64) * 36 + ev.sector.astype(np.int64)) * 4 + np.maximum(ev.leg, 0)
    return np.where(ev.pid >= 0, key, -1)


def match(ev, tracks, hits, min_hits=30, purity=0.9):
    key = segment_keys(ev)
    seg, cnt = np.unique(key[key >= 0], return_counts=True)
    reco = set(seg[cnt >= min_hits].tolist())
    matched = []
    fakes = 0
    for t in tracks:
        h = hits[t["hit_off"]: t["hit_off"] + t["n_hits"]]
        k = key[h]
        u, c = np.unique(k, return_counts=True)
        j = int(np.argmax(c))
        if u[j] >= 0 and c[j] >= purity * len(h):
            matched.append(int(u[j]))
        else:
            matched.append(-1)
            fakes += 1
    found = set(m for m in matched if m in reco)
    n_match_reco = sum(1 for m in matched if m in reco)
    eff = len(found) / max(1, len(reco))
    fake = fakes / max(1, len(tracks))
    clone = (n_match_reco - len(found)) / max(1, len(found))
    return dict(eff=eff, fake=fake, clone=clone, n_reco=len(reco), n_found=len(found),
                n_tracks=len(tracks), matched=np.array(matched, np.int64))


def pulls(ev, tracks, hits):
    """Pulls (fit - truth)/sigma of the five parameters at the innermost hit,
    for tracks matched to a segment whose innermost hit belongs to that same
    segment (truth taken at that cluster's own crossing)."""
    key = segment_keys(ev)
    matched = match(ev, tracks, hits)["matched"]
    out = []
    chi2ndf = []
    for t, mk in zip(tracks, matched):
        h0 = int(t["inner_id"])
        if mk < 0 or key[h0] != mk:
            continue
        tr = ev.truth[h0]
        d = np.array(t["par"]) - tr
        cov = np.array(t["cov"])
        var = cov[[0, 2, 5, 9, 14]]
        out.append(d / np.sqrt(var))
        chi2ndf.append(t["chi2"] / max(1, t["ndf"]))
    return np.array(out), np.array(chi2ndf)
