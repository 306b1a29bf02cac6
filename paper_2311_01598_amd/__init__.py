"""Python binding of the MI355X hybrid key-switching library (libks.so).

Argument marshalling only: every step of the key switch runs in the HIP
kernels behind the C ABI declared in ``include/ks.h``.  PyTorch supplies
device memory and streams; uint32 residues travel in ``torch.int32``
tensors (same bits).  Importing this module loads ``libks.so`` and raises if
it is missing -- there is no fallback path.  With ``KS_LIBRARY=libks_check.so``
in the environment it loads the range-check build instead (the same kernels
with every lazy-range bound tested; ``range_violations`` reads the counts).

The functions keep the C names (``ks_plan_create``, ``ks_keyswitch``, ...);
``Plan`` is a small convenience wrapper around them.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARIES = ("libks.so", "libks_check.so")
_LIB_NAME = os.environ.get("KS_LIBRARY", "libks.so")
if _LIB_NAME not in LIBRARIES:
    raise ImportError(f"KS_LIBRARY={_LIB_NAME!r}: expected one of {LIBRARIES}")
LIB_PATH = os.path.join(HERE, _LIB_NAME)

KS_OK, KS_ERR_INVALID_ARG, KS_ERR_UNSUPPORTED, KS_ERR_NOMEM, KS_ERR_BUDGET, KS_ERR_DEVICE = range(6)
KS_SCHED_AUTO, KS_SCHED_MP, KS_SCHED_DC, KS_SCHED_OC = range(4)
# size of the library's fixed per-GPU array behind ks_keyswitch_noalloc (ks.h)
KS_NOALLOC_SCRATCH_BYTES = 64 << 20
SCHEDULES = {"auto": KS_SCHED_AUTO, "mp": KS_SCHED_MP, "dc": KS_SCHED_DC, "oc": KS_SCHED_OC}


class KsError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {ks_status_string(status)} ({status})")


class ks_params_t(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("num_q", ctypes.c_uint32), ("dnum", ctypes.c_uint32),
                ("num_p", ctypes.c_uint32), ("moduli", ctypes.POINTER(ctypes.c_uint32))]


class ks_config_t(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int), ("tile_towers", ctypes.c_uint32), ("col_width", ctypes.c_uint32),
                ("row_block", ctypes.c_uint32), ("batch_mode", ctypes.c_uint32), ("graph", ctypes.c_uint32),
                ("spin_limit", ctypes.c_uint32), ("batch_order", ctypes.c_uint32)]


class ks_job_t(ctypes.Structure):
    _fields_ = [("evk", ctypes.c_void_p), ("level", ctypes.c_uint32), ("in_", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]


class ks_seeded_job_t(ctypes.Structure):
    _fields_ = [("evk_b", ctypes.c_void_p), ("a_seed", ctypes.c_uint64), ("level", ctypes.c_uint32),
                ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class ks_rotation_t(ctypes.Structure):
    _fields_ = [("evk", ctypes.c_void_p), ("galois", ctypes.c_uint32), ("out", ctypes.c_void_p)]


class ks_seeded_rotation_t(ctypes.Structure):
    _fields_ = [("evk_b", ctypes.c_void_p), ("a_seed", ctypes.c_uint64), ("galois", ctypes.c_uint32),
                ("out", ctypes.c_void_p)]


class ks_rotation_term_t(ctypes.Structure):
    _fields_ = [("evk", ctypes.c_void_p), ("galois", ctypes.c_uint32), ("diag", ctypes.c_void_p)]


class ks_rotate_job_t(ctypes.Structure):
    _fields_ = [("evk", ctypes.c_void_p), ("galois", ctypes.c_uint32), ("level", ctypes.c_uint32),
                ("c0", ctypes.c_void_p), ("c1", ctypes.c_void_p), ("out", ctypes.c_void_p)]


_U32P = ctypes.POINTER(ctypes.c_uint32)
_VP = ctypes.c_void_p
_SIGS = {
    "ks_params_moduli": (ctypes.c_int, [ctypes.POINTER(ks_params_t), _U32P]),
    "ks_root_of_unity": (ctypes.c_uint32, [ctypes.c_uint32, ctypes.c_uint32]),
    "ks_plan_create": (ctypes.c_int, [ctypes.POINTER(ks_params_t), ctypes.POINTER(_VP)]),
    "ks_plan_destroy": (ctypes.c_int, [_VP]),
    "ks_plan_moduli": (ctypes.c_int, [_VP, _U32P]),
    "ks_plan_set_config": (ctypes.c_int, [_VP, ctypes.POINTER(ks_config_t)]),
    "ks_plan_get_config": (ctypes.c_int, [_VP, ctypes.POINTER(ks_config_t)]),
    "ks_oc_work_list": (ctypes.c_int, [ctypes.POINTER(ks_params_t), ctypes.c_uint32, _U32P, _U32P, _U32P, _U32P,
                                       _U32P, _U32P, _U32P]),
    "ks_plan_set_tuned": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(ks_config_t)]),
    "ks_plan_clear_tuned": (ctypes.c_int, [_VP]),
    "ks_plan_resolve_config": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(ks_config_t)]),
    "ks_workspace_size": (ctypes.c_int, [_VP, ctypes.c_uint32, _U32P, ctypes.POINTER(ctypes.c_size_t)]),
    "ks_keyswitch": (ctypes.c_int, [_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "ks_keyswitch_noalloc": (ctypes.c_int, [_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP]),
    "ks_keyswitch_batch": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.POINTER(ks_job_t), _VP, ctypes.c_size_t,
                                          _VP]),
    "ks_keyswitch_seeded": (ctypes.c_int, [_VP, _VP, ctypes.c_uint64, ctypes.c_uint32, _VP, _VP, _VP,
                                           ctypes.c_size_t, _VP]),
    "ks_keyswitch_batch_seeded": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.POINTER(ks_seeded_job_t), _VP,
                                                 ctypes.c_size_t, _VP]),
    "ks_expand_seeded_a": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _VP]),
    "ks_automorphism": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32, _VP, _VP, _VP]),
    "ks_rotate_batch": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.POINTER(ks_rotate_job_t), _VP, ctypes.c_size_t,
                                       _VP]),
    "ks_rotate_workspace_size": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32,
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "ks_rotate_hoisted": (ctypes.c_int, [_VP, ctypes.c_uint32, _VP, _VP, ctypes.c_uint32,
                                         ctypes.POINTER(ks_rotation_t), _VP, ctypes.c_size_t, _VP]),
    "ks_rotate_hoisted_seeded": (ctypes.c_int, [_VP, ctypes.c_uint32, _VP, _VP, ctypes.c_uint32,
                                                ctypes.POINTER(ks_seeded_rotation_t), _VP, ctypes.c_size_t, _VP]),
    "ks_rotate_sum_workspace_size": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32,
                                                    ctypes.POINTER(ctypes.c_size_t)]),
    "ks_rotate_sum_hoisted": (ctypes.c_int, [_VP, ctypes.c_uint32, _VP, _VP, ctypes.c_uint32,
                                             ctypes.POINTER(ks_rotation_term_t), _VP, _VP, ctypes.c_size_t, _VP]),
    "ks_mult_workspace_size": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.POINTER(ctypes.c_size_t)]),
    "ks_mult_relin": (ctypes.c_int, [_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t,
                                     _VP]),
    "ks_batch_status": (ctypes.c_int, [_VP, _VP, _VP, _U32P]),
    "ks_ntt": (ctypes.c_int, [_VP, ctypes.c_uint32, _U32P, ctypes.c_int, _VP, _VP]),
    "ks_trace_enable": (ctypes.c_int, [_VP, ctypes.c_int]),
    "ks_trace_read": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.POINTER(ctypes.c_char_p), _U32P,
                                     ctypes.POINTER(ctypes.c_double), _U32P]),
    "ks_device_rates": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), _VP]),
    "ks_range_violations": (ctypes.c_int, [_U32P, _U32P, ctypes.c_int]),
    "ks_range_set_strict": (ctypes.c_int, [ctypes.c_int]),
    "ks_arith_probe": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, _VP, _VP, _VP, _VP, _VP]),
    "ks_mlp_param_count": (ctypes.c_uint32, [ctypes.c_uint32, ctypes.c_uint32]),
    "ks_mlp_forward": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _VP, _VP, _VP, _VP, _VP]),
    "ks_mlp_mse_grad": (ctypes.c_int, [ctypes.c_uint32, _VP, _VP, _VP, _VP, _VP]),
    "ks_mlp_backward": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _VP, _VP, _VP, _VP, _VP,
                                       _VP, _VP]),
    "ks_mlp_adam": (ctypes.c_int, [ctypes.c_uint32, _VP, _VP, _VP, _VP, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, ctypes.c_uint32, _VP]),
    "ks_status_string": (ctypes.c_char_p, [ctypes.c_int]),
}
EXPORTS = tuple(_SIGS)

# PyTorch ships its own HIP runtime under the same soname as the system one
# libks.so links against.  Loading torch first makes libks.so bind to that
# already-loaded runtime, so the process has exactly one HIP runtime and
# torch's tensors and streams are valid handles for the library.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                      "(hipcc --offload-arch=gfx950).  There is no CPU fallback.")
_lib = ctypes.CDLL(LIB_PATH)
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def lib():
    return _lib


def ks_status_string(status):
    return _lib.ks_status_string(int(status)).decode()


def _check(status, what):
    if status != KS_OK:
        raise KsError(status, what)


def _u32_array(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_uint32 * len(vals))(*vals)


def _params(log_n, num_q, dnum, num_p=0, moduli=None):
    p = ks_params_t(log_n, num_q, dnum, num_p, None)
    keep = None
    if moduli is not None:
        keep = _u32_array(moduli)
        p.moduli = ctypes.cast(keep, _U32P)
    return p, keep


def _ptr(t):
    """Device (or host) address of a tensor / int / None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def ks_params_moduli(log_n, num_q, dnum, num_p=0, moduli=None):
    p, keep = _params(log_n, num_q, dnum, num_p, moduli)
    alpha = -(-num_q // dnum)
    k = num_p or alpha
    out = (ctypes.c_uint32 * (num_q + k))()
    _check(_lib.ks_params_moduli(ctypes.byref(p), out), "ks_params_moduli")
    return list(out)


def ks_root_of_unity(q, log_n):
    return int(_lib.ks_root_of_unity(int(q), int(log_n)))


def ks_plan_create(log_n, num_q, dnum, num_p=0, moduli=None):
    p, keep = _params(log_n, num_q, dnum, num_p, moduli)
    h = _VP()
    _check(_lib.ks_plan_create(ctypes.byref(p), ctypes.byref(h)), "ks_plan_create")
    return h.value


def ks_plan_destroy(plan):
    _check(_lib.ks_plan_destroy(plan), "ks_plan_destroy")


def ks_plan_moduli(plan, count):
    out = (ctypes.c_uint32 * count)()
    _check(_lib.ks_plan_moduli(plan, out), "ks_plan_moduli")
    return list(out)


CONFIG_FIELDS = ("tile_towers", "col_width", "row_block", "batch_mode", "graph", "spin_limit", "batch_order")


def ks_plan_set_config(plan, schedule=0, **fields):
    c = _config(schedule, fields)
    _check(_lib.ks_plan_set_config(plan, ctypes.byref(c)), "ks_plan_set_config")


def ks_plan_get_config(plan):
    c = ks_config_t()
    _check(_lib.ks_plan_get_config(plan, ctypes.byref(c)), "ks_plan_get_config")
    return {"schedule": c.schedule, **{f: getattr(c, f) for f in CONFIG_FIELDS}}


def _config(schedule, fields):
    if isinstance(schedule, str):
        schedule = SCHEDULES[schedule]
    unknown = set(fields) - set(CONFIG_FIELDS)
    if unknown:
        raise TypeError(f"unknown config fields {sorted(unknown)}")
    return ks_config_t(schedule, *[int(fields.get(f, 0)) for f in CONFIG_FIELDS])


def ks_plan_set_tuned(plan, level, count, schedule, **fields):
    c = _config(schedule, fields)
    _check(_lib.ks_plan_set_tuned(plan, int(level), int(count), ctypes.byref(c)), "ks_plan_set_tuned")


def ks_plan_clear_tuned(plan):
    _check(_lib.ks_plan_clear_tuned(plan), "ks_plan_clear_tuned")


def ks_plan_resolve_config(plan, level, count):
    c = ks_config_t()
    _check(_lib.ks_plan_resolve_config(plan, int(level), int(count), ctypes.byref(c)), "ks_plan_resolve_config")
    return {"schedule": c.schedule, **{f: getattr(c, f) for f in CONFIG_FIELDS}}


def ks_batch_status_flag(plan, workspace, stream=None):
    """1 if the last persistent batch in `workspace` hit its spin limit."""
    flag = ctypes.c_uint32()
    _check(_lib.ks_batch_status(plan, _ptr(workspace), _stream(stream), ctypes.byref(flag)), "ks_batch_status")
    return flag.value


def ks_workspace_size(plan, levels):
    n = ctypes.c_size_t()
    arr = _u32_array(levels)
    _check(_lib.ks_workspace_size(plan, len(levels), arr, ctypes.byref(n)), "ks_workspace_size")
    return n.value


def ks_keyswitch(plan, evk, level, inp, out, workspace, workspace_bytes=None, stream=None):
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    st = _lib.ks_keyswitch(plan, _ptr(evk), int(level), _ptr(inp), _ptr(out), _ptr(workspace),
                           int(workspace_bytes), _stream(stream))
    _check(st, "ks_keyswitch")


def ks_keyswitch_noalloc(plan, evk, level, inp, out, stream=None):
    st = _lib.ks_keyswitch_noalloc(plan, _ptr(evk), int(level), _ptr(inp), _ptr(out), _stream(stream))
    _check(st, "ks_keyswitch_noalloc")


def ks_keyswitch_batch(plan, jobs, workspace, workspace_bytes=None, stream=None):
    """jobs: list of (evk, level, in, out) tensors/addresses."""
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    arr = (ks_job_t * len(jobs))()
    for i, (evk, level, inp, out) in enumerate(jobs):
        arr[i] = ks_job_t(_ptr(evk), int(level), _ptr(inp), _ptr(out))
    st = _lib.ks_keyswitch_batch(plan, len(jobs), arr, _ptr(workspace), int(workspace_bytes), _stream(stream))
    _check(st, "ks_keyswitch_batch")


def ks_keyswitch_seeded(plan, evk_b, a_seed, level, inp, out, workspace, workspace_bytes=None, stream=None):
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    st = _lib.ks_keyswitch_seeded(plan, _ptr(evk_b), int(a_seed) & (2**64 - 1), int(level), _ptr(inp), _ptr(out),
                                  _ptr(workspace), int(workspace_bytes), _stream(stream))
    _check(st, "ks_keyswitch_seeded")


def ks_keyswitch_batch_seeded(plan, jobs, workspace, workspace_bytes=None, stream=None):
    """jobs: list of (evk_b, a_seed, level, in, out)."""
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    arr = (ks_seeded_job_t * len(jobs))()
    for i, (evk_b, a_seed, level, inp, out) in enumerate(jobs):
        arr[i] = ks_seeded_job_t(_ptr(evk_b), int(a_seed) & (2**64 - 1), int(level), _ptr(inp), _ptr(out))
    st = _lib.ks_keyswitch_batch_seeded(plan, len(jobs), arr, _ptr(workspace), int(workspace_bytes),
                                        _stream(stream))
    _check(st, "ks_keyswitch_batch_seeded")


def ks_expand_seeded_a(plan, a_seed, evk, stream=None):
    _check(_lib.ks_expand_seeded_a(plan, int(a_seed) & (2**64 - 1), _ptr(evk), _stream(stream)),
           "ks_expand_seeded_a")


def ks_automorphism(plan, galois, count, inp, out, stream=None):
    _check(_lib.ks_automorphism(plan, int(galois), int(count), _ptr(inp), _ptr(out), _stream(stream)),
           "ks_automorphism")


def ks_rotate_batch(plan, jobs, workspace, workspace_bytes=None, stream=None):
    """jobs: list of (evk, galois, level, c0, c1, out)."""
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    arr = (ks_rotate_job_t * max(len(jobs), 1))()
    for i, (evk, galois, level, c0, c1, out) in enumerate(jobs):
        arr[i] = ks_rotate_job_t(_ptr(evk), int(galois), int(level), _ptr(c0), _ptr(c1), _ptr(out))
    _check(_lib.ks_rotate_batch(plan, len(jobs), arr, _ptr(workspace), int(workspace_bytes), _stream(stream)),
           "ks_rotate_batch")


def ks_rotate_workspace_size(plan, level, count):
    n = ctypes.c_size_t(0)
    _check(_lib.ks_rotate_workspace_size(plan, int(level), int(count), ctypes.byref(n)), "ks_rotate_workspace_size")
    return n.value


def ks_rotate_hoisted(plan, level, c0, c1, rots, workspace, workspace_bytes=None, stream=None):
    """rots: list of (evk, galois, out)."""
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    arr = (ks_rotation_t * max(len(rots), 1))()
    for i, (evk, galois, out) in enumerate(rots):
        arr[i] = ks_rotation_t(_ptr(evk), int(galois), _ptr(out))
    _check(_lib.ks_rotate_hoisted(plan, int(level), _ptr(c0), _ptr(c1), len(rots), arr, _ptr(workspace),
                                  int(workspace_bytes), _stream(stream)), "ks_rotate_hoisted")


def ks_rotate_hoisted_seeded(plan, level, c0, c1, rots, workspace, workspace_bytes=None, stream=None):
    """rots: list of (evk_b, a_seed, galois, out)."""
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    arr = (ks_seeded_rotation_t * max(len(rots), 1))()
    for i, (evk_b, a_seed, galois, out) in enumerate(rots):
        arr[i] = ks_seeded_rotation_t(_ptr(evk_b), int(a_seed) & (2**64 - 1), int(galois), _ptr(out))
    _check(_lib.ks_rotate_hoisted_seeded(plan, int(level), _ptr(c0), _ptr(c1), len(rots), arr, _ptr(workspace),
                                         int(workspace_bytes), _stream(stream)), "ks_rotate_hoisted_seeded")


def ks_rotate_sum_workspace_size(plan, level, count):
    n = ctypes.c_size_t(0)
    _check(_lib.ks_rotate_sum_workspace_size(plan, int(level), int(count), ctypes.byref(n)),
           "ks_rotate_sum_workspace_size")
    return n.value


def ks_rotate_sum_hoisted(plan, level, c0, c1, terms, out, workspace, workspace_bytes=None, stream=None):
    """terms: list of (evk, galois, diag or None)."""
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    arr = (ks_rotation_term_t * max(len(terms), 1))()
    for i, (evk, galois, diag) in enumerate(terms):
        arr[i] = ks_rotation_term_t(_ptr(evk), int(galois), _ptr(diag) if diag is not None else None)
    _check(_lib.ks_rotate_sum_hoisted(plan, int(level), _ptr(c0), _ptr(c1), len(terms), arr, _ptr(out),
                                      _ptr(workspace), int(workspace_bytes), _stream(stream)), "ks_rotate_sum_hoisted")


def ks_mult_workspace_size(plan, level):
    n = ctypes.c_size_t(0)
    _check(_lib.ks_mult_workspace_size(plan, int(level), ctypes.byref(n)), "ks_mult_workspace_size")
    return n.value


def ks_mult_relin(plan, evk, level, a0, a1, b0, b1, out, workspace, workspace_bytes=None, stream=None):
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    _check(_lib.ks_mult_relin(plan, _ptr(evk), int(level), _ptr(a0), _ptr(a1), _ptr(b0), _ptr(b1), _ptr(out),
                              _ptr(workspace), int(workspace_bytes), _stream(stream)), "ks_mult_relin")


def galois_rotation(log_n, r):
    """Galois element of a rotation by r slots: 5^r mod 2N."""
    two_n = 2 << log_n
    return pow(5, r % (two_n // 4), two_n)


def ks_ntt(plan, g, inverse, data, stream=None):
    arr = _u32_array(g)
    _check(_lib.ks_ntt(plan, len(g), arr, int(bool(inverse)), _ptr(data), _stream(stream)), "ks_ntt")


def ks_trace_enable(plan, on=True):
    _check(_lib.ks_trace_enable(plan, int(bool(on))), "ks_trace_enable")


def ks_trace_read(plan, max_names=64):
    """{stage name: (launches, total ms)} recorded since the last read."""
    names = (ctypes.c_char_p * max_names)()
    launches = (ctypes.c_uint32 * max_names)()
    ms = (ctypes.c_double * max_names)()
    count = ctypes.c_uint32()
    _check(_lib.ks_trace_read(plan, max_names, names, launches, ms, ctypes.byref(count)), "ks_trace_read")
    return {names[i].decode(): (launches[i], ms[i]) for i in range(min(count.value, max_names))}


RATE_NAMES = ("add_u32", "mul_lo_u32", "mul_hi_u32", "mad_u64_u32", "fma_f64", "copy_bytes", "butterfly")


def ks_device_rates(stream=None):
    out = (ctypes.c_double * 7)()
    _check(_lib.ks_device_rates(out, _stream(stream)), "ks_device_rates")
    return dict(zip(RATE_NAMES, list(out)))


def ks_range_violations(reset=False):
    """(count, code): range-check violations on the current device since the
    last reset (range-check build only; the normal build raises KsError with
    KS_ERR_UNSUPPORTED)."""
    count, code = ctypes.c_uint32(0), ctypes.c_uint32(0)
    _check(_lib.ks_range_violations(ctypes.byref(count), ctypes.byref(code), 1 if reset else 0),
           "ks_range_violations")
    return int(count.value), int(code.value)


def ks_range_set_strict(on):
    _check(_lib.ks_range_set_strict(1 if on else 0), "ks_range_set_strict")


def ks_arith_probe(q, a, b, w, out=None, stream=None):
    """The 30-bit primitives on int32 device tensors a, b, w of n words;
    returns out [n][8] (see include/ks.h)."""
    import torch
    n = a.numel()
    if out is None:
        out = torch.empty((n, 8), dtype=torch.int32, device=a.device)
    _check(_lib.ks_arith_probe(int(q), n, _ptr(a), _ptr(b), _ptr(w), _ptr(out), _stream(stream)), "ks_arith_probe")
    return out


def ks_mlp_param_count(F, H):
    return int(_lib.ks_mlp_param_count(F, H))


def ks_mlp_forward(F, H, B, params, X, Y, act, stream=None):
    _check(_lib.ks_mlp_forward(F, H, B, _ptr(params), _ptr(X), _ptr(Y), _ptr(act), _stream(stream)),
           "ks_mlp_forward")


def ks_mlp_mse_grad(B, Y, T, dY, loss, stream=None):
    _check(_lib.ks_mlp_mse_grad(B, _ptr(Y), _ptr(T), _ptr(dY), _ptr(loss), _stream(stream)), "ks_mlp_mse_grad")


def ks_mlp_backward(F, H, B, params, X, act, dY, grads, scratch, stream=None):
    _check(_lib.ks_mlp_backward(F, H, B, _ptr(params), _ptr(X), _ptr(act), _ptr(dY), _ptr(grads), _ptr(scratch),
                                _stream(stream)), "ks_mlp_backward")


def ks_mlp_adam(n, params, grads, m, v, lr, beta1, beta2, eps, step, stream=None):
    _check(_lib.ks_mlp_adam(n, _ptr(params), _ptr(grads), _ptr(m), _ptr(v), lr, beta1, beta2, eps, step,
                            _stream(stream)), "ks_mlp_adam")


class Plan:
    """A key-switching plan on the current device (owns the C handle)."""

    def __init__(self, log_n, num_q, dnum, num_p=0, moduli=None, schedule=None, **cfg):
        self.log_n, self.num_q, self.dnum = log_n, num_q, dnum
        self.alpha = -(-num_q // dnum)
        self.num_p = num_p or self.alpha
        self.n = 1 << log_n
        self.handle = ks_plan_create(log_n, num_q, dnum, num_p, moduli)
        self.moduli = ks_plan_moduli(self.handle, num_q + self.num_p)
        if schedule is not None or cfg:
            self.configure(schedule or 0, **cfg)

    def configure(self, schedule=0, **fields):
        ks_plan_set_config(self.handle, schedule, **fields)

    def set_tuned(self, level, count, schedule, **fields):
        """Record the tuner's configuration for calls of `count` key switches
        whose largest level is `level` (used while the schedule is "auto")."""
        ks_plan_set_tuned(self.handle, level, count, schedule, **fields)

    def clear_tuned(self):
        ks_plan_clear_tuned(self.handle)

    def resolve(self, level, count=1):
        """The configuration a call of that shape runs with."""
        return ks_plan_resolve_config(self.handle, level, count)

    @property
    def config(self):
        return ks_plan_get_config(self.handle)

    def workspace_bytes(self, levels):
        return ks_workspace_size(self.handle, list(levels))

    def workspace(self, levels, device="cuda"):
        import torch
        nbytes = max(self.workspace_bytes(levels), 256)
        return torch.empty((nbytes + 3) // 4, dtype=torch.int32, device=device)

    def keyswitch(self, evk, level, d, out=None, workspace=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((2, level + 1, self.n), dtype=torch.int32, device=d.device)
        if workspace is None:
            workspace = self.workspace([level], d.device)
        ks_keyswitch(self.handle, evk, level, d, out, workspace, stream=stream)
        return out

    def keyswitch_batch(self, jobs, workspace=None, stream=None, workspace_bytes=None):
        if workspace is None:
            workspace = self.workspace([j[1] for j in jobs])
        ks_keyswitch_batch(self.handle, jobs, workspace, workspace_bytes, stream=stream)

    def keyswitch_seeded(self, evk_b, a_seed, level, d, out=None, workspace=None, stream=None):
        """Key switch with a compressed key: evk_b [dnum][L+1+K][N] plus the
        seed of the a halves (Sec. IV-D)."""
        import torch
        if out is None:
            out = torch.empty((2, level + 1, self.n), dtype=torch.int32, device=d.device)
        if workspace is None:
            workspace = self.workspace([level], d.device)
        ks_keyswitch_seeded(self.handle, evk_b, a_seed, level, d, out, workspace, stream=stream)
        return out

    def keyswitch_batch_seeded(self, jobs, workspace=None, stream=None, workspace_bytes=None):
        if workspace is None:
            workspace = self.workspace([j[2] for j in jobs])
        ks_keyswitch_batch_seeded(self.handle, jobs, workspace, workspace_bytes, stream=stream)

    def expand_seeded_a(self, a_seed, evk, stream=None):
        ks_expand_seeded_a(self.handle, a_seed, evk, stream=stream)

    def _ws(self, nbytes, device):
        import torch
        return torch.empty((max(nbytes, 256) + 3) // 4, dtype=torch.int32, device=device)

    def automorphism(self, x, galois, out=None, stream=None):
        """Evaluation-domain automorphism X -> X^galois of every limb of x."""
        import torch
        if out is None:
            out = torch.empty_like(x)
        ks_automorphism(self.handle, galois, x.numel() // self.n, x, out, stream=stream)
        return out

    def rotate_hoisted(self, level, c0, c1, rots, workspace=None, stream=None):
        """rots: list of (evk, galois); returns the rotated ciphertexts
        [2][level+1][N], one per rotation, sharing one ModUp of c1."""
        import torch
        outs = [torch.empty((2, level + 1, self.n), dtype=torch.int32, device=c1.device) for _ in rots]
        if workspace is None:
            workspace = self._ws(ks_rotate_workspace_size(self.handle, level, len(rots)), c1.device)
        ks_rotate_hoisted(self.handle, level, c0, c1, [(e, g, o) for (e, g), o in zip(rots, outs)], workspace,
                          stream=stream)
        return outs

    def rotate_hoisted_seeded(self, level, c0, c1, rots, workspace=None, stream=None):
        """rots: list of (evk_b, a_seed, galois) with compressed keys."""
        import torch
        outs = [torch.empty((2, level + 1, self.n), dtype=torch.int32, device=c1.device) for _ in rots]
        if workspace is None:
            workspace = self._ws(ks_rotate_workspace_size(self.handle, level, len(rots)), c1.device)
        ks_rotate_hoisted_seeded(self.handle, level, c0, c1, [(e, a, g, o) for (e, a, g), o in zip(rots, outs)],
                                 workspace, stream=stream)
        return outs

    def rotate_sum_hoisted(self, level, c0, c1, terms, out=None, workspace=None, stream=None):
        """terms: list of (evk, galois, diag or None); returns
        sum_r diag_r * sigma_r((c0, c1)) with one ModUp and one ModDown."""
        import torch
        if out is None:
            out = torch.empty((2, level + 1, self.n), dtype=torch.int32, device=c1.device)
        if workspace is None:
            workspace = self._ws(ks_rotate_sum_workspace_size(self.handle, level, len(terms)), c1.device)
        ks_rotate_sum_hoisted(self.handle, level, c0, c1, terms, out, workspace, stream=stream)
        return out

    def rotate_batch(self, jobs, workspace=None, stream=None):
        """jobs: list of (evk, galois, level, c0, c1); returns one rotated
        ciphertext per job, all in one launch per phase."""
        import torch
        outs = [torch.empty((2, j[2] + 1, self.n), dtype=torch.int32, device=j[4].device) for j in jobs]
        if workspace is None:
            workspace = self.workspace([j[2] for j in jobs])
        ks_rotate_batch(self.handle, [tuple(j) + (o,) for j, o in zip(jobs, outs)], workspace, stream=stream)
        return outs

    def rotate(self, evk, galois, level, c0, c1, workspace=None, stream=None):
        return self.rotate_hoisted(level, c0, c1, [(evk, galois)], workspace, stream)[0]

    def mult_relin(self, evk, level, a0, a1, b0, b1, out=None, workspace=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((2, level + 1, self.n), dtype=torch.int32, device=a0.device)
        if workspace is None:
            workspace = self._ws(ks_mult_workspace_size(self.handle, level), a0.device)
        ks_mult_relin(self.handle, evk, level, a0, a1, b0, b1, out, workspace, stream=stream)
        return out

    def ntt(self, data, g, inverse=False, stream=None):
        ks_ntt(self.handle, list(g), inverse, data, stream=stream)

    def close(self):
        if self.handle:
            ks_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- 64-bit words
class ks64_params_t(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("num_q", ctypes.c_uint32), ("dnum", ctypes.c_uint32),
                ("num_p", ctypes.c_uint32), ("moduli", ctypes.POINTER(ctypes.c_uint64))]


_U64P = ctypes.POINTER(ctypes.c_uint64)
_SIGS64 = {
    "ks64_params_moduli": (ctypes.c_int, [ctypes.POINTER(ks64_params_t), _U64P]),
    "ks64_root_of_unity": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint32]),
    "ks64_plan_create": (ctypes.c_int, [ctypes.POINTER(ks64_params_t), ctypes.POINTER(_VP)]),
    "ks64_plan_destroy": (ctypes.c_int, [_VP]),
    "ks64_plan_moduli": (ctypes.c_int, [_VP, _U64P]),
    "ks64_workspace_size": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.POINTER(ctypes.c_size_t)]),
    "ks64_keyswitch": (ctypes.c_int, [_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "ks64_ntt": (ctypes.c_int, [_VP, ctypes.c_uint32, _U32P, ctypes.c_int, _VP, _VP]),
    "ks64_arith_probe": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, _VP, _VP, _VP, _VP]),
    "ks64_keyswitch_seeded": (ctypes.c_int, [_VP, _VP, ctypes.c_uint64, ctypes.c_uint32, _VP, _VP, _VP,
                                             ctypes.c_size_t, _VP]),
}
for _name, (_res, _args) in _SIGS64.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
EXPORTS = EXPORTS + tuple(_SIGS64)


def _params64(log_n, num_q, dnum, num_p=0, moduli=None):
    p = ks64_params_t(log_n, num_q, dnum, num_p, None)
    keep = None
    if moduli is not None:
        keep = (ctypes.c_uint64 * len(moduli))(*[int(m) for m in moduli])
        p.moduli = ctypes.cast(keep, _U64P)
    return p, keep


def ks64_params_moduli(log_n, num_q, dnum, num_p=0, moduli=None):
    p, keep = _params64(log_n, num_q, dnum, num_p, moduli)
    alpha = -(-num_q // dnum)
    out = (ctypes.c_uint64 * (num_q + (num_p or alpha)))()
    _check(_lib.ks64_params_moduli(ctypes.byref(p), out), "ks64_params_moduli")
    return list(out)


def ks64_root_of_unity(q, log_n):
    return int(_lib.ks64_root_of_unity(int(q), int(log_n)))


def ks64_plan_create(log_n, num_q, dnum, num_p=0, moduli=None):
    p, keep = _params64(log_n, num_q, dnum, num_p, moduli)
    h = _VP()
    _check(_lib.ks64_plan_create(ctypes.byref(p), ctypes.byref(h)), "ks64_plan_create")
    return h.value


def ks64_plan_destroy(plan):
    _check(_lib.ks64_plan_destroy(plan), "ks64_plan_destroy")


def ks64_workspace_size(plan, level):
    b = ctypes.c_size_t()
    _check(_lib.ks64_workspace_size(plan, int(level), ctypes.byref(b)), "ks64_workspace_size")
    return b.value


def ks64_keyswitch(plan, evk, level, inp, out, workspace, workspace_bytes=None, stream=None):
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    st = _lib.ks64_keyswitch(plan, _ptr(evk), int(level), _ptr(inp), _ptr(out), _ptr(workspace),
                             int(workspace_bytes), _stream(stream))
    _check(st, "ks64_keyswitch")


def ks64_keyswitch_seeded(plan, evk_b, a_seed, level, inp, out, workspace, workspace_bytes=None, stream=None):
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size()
    st = _lib.ks64_keyswitch_seeded(plan, _ptr(evk_b), int(a_seed) & 0xFFFFFFFFFFFFFFFF, int(level), _ptr(inp),
                                    _ptr(out), _ptr(workspace), int(workspace_bytes), _stream(stream))
    _check(st, "ks64_keyswitch_seeded")


def ks64_arith_probe(q, w, a, b, out=None, stream=None):
    """The 64-bit primitives on int64 device tensors a, b of n words with
    the twiddle w; returns out [n][9] (see include/ks.h)."""
    import torch
    n = a.numel()
    if out is None:
        out = torch.empty((n, 9), dtype=torch.int64, device=a.device)
    _check(_lib.ks64_arith_probe(int(q), int(w), n, _ptr(a), _ptr(b), _ptr(out), _stream(stream)),
           "ks64_arith_probe")
    return out


def ks64_ntt(plan, g, inverse, data, stream=None):
    g = list(g)
    arr = (ctypes.c_uint32 * max(1, len(g)))(*g)
    _check(_lib.ks64_ntt(plan, len(g), arr, 1 if inverse else 0, _ptr(data), _stream(stream)), "ks64_ntt")


class Plan64:
    """A 64-bit-word key-switching plan on the current device (uint64
    residues travel in torch.int64 tensors, same bits)."""

    def __init__(self, log_n, num_q, dnum, num_p=0, moduli=None):
        self.log_n, self.num_q, self.dnum = log_n, num_q, dnum
        self.alpha = -(-num_q // dnum)
        self.num_p = num_p or self.alpha
        self.n = 1 << log_n
        self.handle = ks64_plan_create(log_n, num_q, dnum, num_p, moduli)
        out = (ctypes.c_uint64 * (num_q + self.num_p))()
        _check(_lib.ks64_plan_moduli(self.handle, out), "ks64_plan_moduli")
        self.moduli = list(out)

    def workspace(self, level, device="cuda"):
        import torch
        return torch.empty((ks64_workspace_size(self.handle, level) + 7) // 8, dtype=torch.int64, device=device)

    def keyswitch(self, evk, level, d, out=None, workspace=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((2, level + 1, self.n), dtype=torch.int64, device=d.device)
        if workspace is None:
            workspace = self.workspace(level, d.device)
        ks64_keyswitch(self.handle, evk, level, d, out, workspace, stream=stream)
        return out

    def keyswitch_seeded(self, evk_b, a_seed, level, d, out=None, workspace=None, stream=None):
        """Key switch with a compressed key: evk_b [dnum][L+1+K][N] holds the b
        halves, the a halves are regenerated from a_seed on the device."""
        import torch
        if out is None:
            out = torch.empty((2, level + 1, self.n), dtype=torch.int64, device=d.device)
        if workspace is None:
            workspace = self.workspace(level, d.device)
        ks64_keyswitch_seeded(self.handle, evk_b, a_seed, level, d, out, workspace, stream=stream)
        return out

    def ntt(self, data, g, inverse=False, stream=None):
        ks64_ntt(self.handle, g, inverse, data, stream)

    def close(self):
        if self.handle:
            ks64_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
