"""MI355X channel-flow DNS environment (HIP/gfx950) behind a C ABI.

The numerical work runs in ``libchanenv.so`` (built from ``csrc/`` by
``build.py``); :mod:`.binding` marshals arguments to it.  There is no CPU path:
if the library is missing, loading fails loudly.
"""
from .binding import (ChanEnv, ChanGrid, ChanInfo, ChanOpts, ChanError, chan_env_create,
                      chan_env_destroy, chan_env_footprint_bytes, chan_env_get_state,
                      chan_env_query, chan_env_reset, chan_env_set_state, chan_env_set_timing,
                      chan_env_step, chan_env_timing_read, chan_kernel_class_name, chan_last_error,
                      chan_opts_default, chan_strerror, library_path, load_library)

__all__ = ["ChanEnv", "ChanGrid", "ChanInfo", "ChanOpts", "ChanError", "chan_env_create",
           "chan_env_destroy", "chan_env_footprint_bytes", "chan_env_get_state",
           "chan_env_query", "chan_env_reset", "chan_env_set_state", "chan_env_set_timing",
           "chan_env_step", "chan_env_timing_read", "chan_kernel_class_name",
           "chan_last_error", "chan_opts_default", "chan_strerror", "library_path", "load_library"]
