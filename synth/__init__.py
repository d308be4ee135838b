"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  Holds no step of the processing method itself."""
from .vmi import (GRID, KIND_OTHER, KIND_PIXEL, KIND_TRIGGER, PIX_WRAP_TICKS,  # noqa: F401
                  SHOT_PERIOD_TICKS, SPECS, TDC_WRAP_TICKS, TICK_NS, TRIG_SUBTYPE,
                  Spec, Workload, encode_pixels, encode_tdc, generate, make_config,
                  tiny_events)
from .clusters import init_mlp_params, make_clusters  # noqa: F401,E402
from .walkcal import WALK_DEFAULT, calibration_run, walk_ns  # noqa: F401,E402
