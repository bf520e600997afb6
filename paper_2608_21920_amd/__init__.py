"""MI355X-native per-step particle loop of the 1D radiative PIC of pulsar
polar-cap pair discharges: a HIP library (libgap.so) behind a C ABI, with a
thin ctypes binding."""
from .gap import Gap, GapError, GapParams, load_library, sync_inverse_host, window_loss, FLAGS  # noqa: F401
from . import workloads  # noqa: F401
