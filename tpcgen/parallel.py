"""Generate many synthetic events in worker processes (spawned, so it is
safe before or after the parent touches the GPU).  Workers return only the
cluster arrays (sector, row, y, z) and the error model."""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

from . import events as E


def _one(spec):
    kind, args = spec
    fn = {"pp": E.pp_event, "pbpb": E.pbpb_event, "central": E.central_event,
          "batch": E.batch_event, "one_sector": E.one_sector_event}[kind]
    ev = fn(*args)
    return dict(name=ev.name, sector=ev.sector, row=ev.row, y=ev.y, z=ev.z, sigma=ev.sigma)


def generate(specs, workers: int | None = None):
    """specs: list of (kind, args) with kind in pp, pbpb, central, batch,
    one_sector.  Returns a list of dicts in the same order."""
    workers = workers or min(16, os.cpu_count() or 1, max(1, len(specs)))
    if workers <= 1:
        return [_one(s) for s in specs]
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_one, specs))
