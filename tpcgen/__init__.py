"""Seeded synthetic TPC events and the detector description (inputs only)."""
from . import geometry
from .events import (Event, one_sector_event, pp_event, pbpb_event, central_event,
                     batch_multiplicities, batch_event, serve_event, seed_for,
                     tiny_event, distort_drift, drift_z, membrane_event,
                     boundary_jet_event)

__all__ = ["geometry", "Event", "one_sector_event", "pp_event", "pbpb_event",
           "central_event", "batch_multiplicities", "batch_event", "serve_event",
           "seed_for", "tiny_event", "distort_drift", "drift_z", "membrane_event",
           "boundary_jet_event"]
