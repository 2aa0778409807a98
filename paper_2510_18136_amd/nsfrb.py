"""ctypes binding of the C ABI in include/nsfrb.h (argument marshalling only).

Every step of the search runs in the HIP library libnsfrb.so. PyTorch, when
used by a caller, only provides device buffers and streams: pass
`tensor.data_ptr()` and `torch.cuda.current_stream().cuda_stream`.
Loading fails loudly when the library has not been built. A process that
uses both should import torch and touch its device (torch.cuda.is_available())
before the first library call, so that both share the HIP runtime torch loads.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libnsfrb.so")

OK, INVALID_ARG, UNSUPPORTED, OUT_OF_MEMORY, DEVICE, NOT_READY, TRUNCATED = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "OUT_OF_MEMORY",
                4: "DEVICE", 5: "NOT_READY", 6: "TRUNCATED"}
DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
DTYPE_BYTES = {"f32": 4, "f16": 2, "bf16": 2}
NORMS = {"pixel_subband": 0, "external": 2, "none": 3}
LAYOUTS = {"tsp": 0, "pst": 1}

# every symbol declared in include/nsfrb.h
EXPORTS = [
    "nsfrb_version", "nsfrb_last_error", "nsfrb_config_validate", "nsfrb_plan_delays",
    "nsfrb_search_create", "nsfrb_search_destroy", "nsfrb_search_run", "nsfrb_candidates_get",
    "nsfrb_delay_table_get", "nsfrb_maps_get", "nsfrb_best_get", "nsfrb_noise_stats_get",
    "nsfrb_noise_stats_set", "nsfrb_zcube_get", "nsfrb_zcube_device", "nsfrb_flag_count_get", "nsfrb_maps_device",
    "nsfrb_profiling_enable", "nsfrb_stage_times_get", "nsfrb_search_plan_info",
    "nsfrb_batch_create", "nsfrb_batch_destroy", "nsfrb_batch_run", "nsfrb_batch_run_separate",
    "nsfrb_batch_use_graph", "nsfrb_batch_candidates_get", "nsfrb_batch_maps_get", "nsfrb_batch_best_get",
    "nsfrb_batch_zcube_device", "nsfrb_batch_info_get",
    "nsfrb_generate_noise", "nsfrb_inject_boxcar", "nsfrb_inject_boxcars", "nsfrb_inject_boxcars_static", "nsfrb_philox_fill", "nsfrb_inject_rfi",
    "nsfrb_classifier_param_count", "nsfrb_classifier_create", "nsfrb_classifier_destroy",
    "nsfrb_classifier_params_get", "nsfrb_classifier_params_set", "nsfrb_classifier_set_lr",
    "nsfrb_classifier_grads_get", "nsfrb_classifier_state_bytes", "nsfrb_classifier_save", "nsfrb_classifier_load",
    "nsfrb_classifier_activations_get", "nsfrb_classifier_grad_pre_get", "nsfrb_classifier_logits_get",
    "nsfrb_classifier_train_step", "nsfrb_classifier_infer", "nsfrb_cutouts_extract",
    "nsfrb_bin_time", "nsfrb_multiscale_create", "nsfrb_multiscale_destroy", "nsfrb_multiscale_run",
    "nsfrb_multiscale_scale", "nsfrb_multiscale_candidates_get", "nsfrb_plan_dm_grid",
    "nsfrb_psf_reduce", "nsfrb_stream_create", "nsfrb_stream_destroy", "nsfrb_stream_push", "nsfrb_stream_search",
]


class Config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("n_sub", ctypes.c_int32), ("n_time", ctypes.c_int32),
        ("freq_ghz", ctypes.POINTER(ctypes.c_double)),
        ("f_ref_ghz", ctypes.c_double), ("dt_ms", ctypes.c_double), ("k_dm_ms", ctypes.c_double),
        ("n_dm", ctypes.c_int32), ("dm", ctypes.POINTER(ctypes.c_double)),
        ("n_width", ctypes.c_int32), ("width", ctypes.POINTER(ctypes.c_int32)),
        ("in_dtype", ctypes.c_int32), ("store_dtype", ctypes.c_int32), ("norm", ctypes.c_int32),
        ("snr_threshold", ctypes.c_float), ("max_candidates", ctypes.c_int32),
        ("device", ctypes.c_int32), ("layout", ctypes.c_int32),
    ]


class Candidate(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int32), ("y", ctypes.c_int32), ("dm_index", ctypes.c_int32),
                ("width_index", ctypes.c_int32), ("toa", ctypes.c_int32), ("snr", ctypes.c_float)]


class ScaleCandidate(ctypes.Structure):
    _fields_ = [("cand", Candidate), ("scale", ctypes.c_int32)]


class StreamResult(ctypes.Structure):
    _fields_ = [("searched", ctypes.c_int32), ("has_candidate", ctypes.c_int32), ("cand", Candidate),
                ("chunk_index", ctypes.c_int64), ("window_start", ctypes.c_int64), ("search_ms", ctypes.c_float),
                ("dropped_total", ctypes.c_int32), ("flagged", ctypes.c_int64)]


class ClassifierConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_batch", ctypes.c_int32), ("n_time", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("device", ctypes.c_int32)]


class Boxcar(ctypes.Structure):
    _fields_ = [("cube", ctypes.c_int32), ("pixel", ctypes.c_int32), ("t0", ctypes.c_int32),
                ("width", ctypes.c_int32), ("amp", ctypes.c_float)]


class CutoutDesc(ctypes.Structure):
    _fields_ = [("cube", ctypes.c_int64), ("px", ctypes.c_int32), ("py", ctypes.c_int32),
                ("dm_index", ctypes.c_int32), ("toa", ctypes.c_int32)]


class NsfrbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libnsfrb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, pi32 = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)
        pd, pf = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)
        sig = {
            "nsfrb_version": ([], ctypes.c_char_p),
            "nsfrb_last_error": ([], ctypes.c_char_p),
            "nsfrb_config_validate": ([ctypes.POINTER(Config)], ctypes.c_int),
            "nsfrb_plan_delays": ([ctypes.POINTER(Config), pi32], ctypes.c_int),
            "nsfrb_search_create": ([ctypes.POINTER(Config), ctypes.POINTER(vp)], ctypes.c_int),
            "nsfrb_search_destroy": ([vp], ctypes.c_int),
            "nsfrb_search_run": ([vp, vp, vp], ctypes.c_int),
            "nsfrb_candidates_get": ([vp, ctypes.POINTER(Candidate), i32, pi32, pi32], ctypes.c_int),
            "nsfrb_delay_table_get": ([vp, pi32], ctypes.c_int),
            "nsfrb_maps_get": ([vp, pf, pi32], ctypes.c_int),
            "nsfrb_best_get": ([vp, pf, pi32, pi32, pi32], ctypes.c_int),
            "nsfrb_noise_stats_get": ([vp, pd, pd], ctypes.c_int),
            "nsfrb_noise_stats_set": ([vp, pd, pd], ctypes.c_int),
            "nsfrb_zcube_get": ([vp, vp], ctypes.c_int),
            "nsfrb_zcube_device": ([vp, ctypes.POINTER(vp)], ctypes.c_int),
            "nsfrb_flag_count_get": ([vp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
            "nsfrb_maps_device": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp)], ctypes.c_int),
            "nsfrb_profiling_enable": ([vp, i32], ctypes.c_int),
            "nsfrb_stage_times_get": ([vp, pf], ctypes.c_int),
            "nsfrb_debug_plan_source": ([ctypes.POINTER(Config), ctypes.c_char_p, i32, i32], ctypes.c_int),
            "nsfrb_search_plan_info": ([vp, pi32], ctypes.c_int),
            "nsfrb_batch_create": ([ctypes.POINTER(Config), i32, ctypes.POINTER(vp)], ctypes.c_int),
            "nsfrb_batch_destroy": ([vp], ctypes.c_int),
            "nsfrb_batch_run": ([vp, ctypes.POINTER(vp), vp], ctypes.c_int),
            "nsfrb_batch_run_separate": ([vp, ctypes.POINTER(vp), vp], ctypes.c_int),
            "nsfrb_batch_use_graph": ([vp, i32], ctypes.c_int),
            "nsfrb_batch_candidates_get": ([vp, i32, ctypes.POINTER(Candidate), i32, pi32, pi32], ctypes.c_int),
            "nsfrb_batch_maps_get": ([vp, i32, pf, pi32], ctypes.c_int),
            "nsfrb_batch_best_get": ([vp, i32, pf, pi32, pi32, pi32], ctypes.c_int),
            "nsfrb_batch_zcube_device": ([vp, i32, ctypes.POINTER(vp)], ctypes.c_int),
            "nsfrb_batch_info_get": ([vp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
            "nsfrb_generate_noise": ([vp, i32, i32, i32, i32, i32, ctypes.c_uint64, ctypes.c_float, vp],
                                     ctypes.c_int),
            "nsfrb_inject_boxcar": ([vp, i32, i32, i32, i32, i32, i32, i32, i32, ctypes.c_float, pi32, vp],
                                    ctypes.c_int),
            "nsfrb_inject_boxcars": ([ctypes.POINTER(vp), i32, i32, i32, i32, i32, i32, ctypes.POINTER(Boxcar),
                                      pi32, i32, vp], ctypes.c_int),
            "nsfrb_inject_boxcars_static": ([ctypes.POINTER(vp), i32, i32, i32, i32, i32, i32,
                                             ctypes.POINTER(Boxcar), pi32, i32, vp], ctypes.c_int),
            "nsfrb_philox_fill": ([vp, ctypes.c_int64, ctypes.c_uint64, vp], ctypes.c_int),
            "nsfrb_classifier_state_bytes": ([], ctypes.c_int64),
            "nsfrb_classifier_save": ([vp, ctypes.c_uint64, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)],
                                      ctypes.c_int),
            "nsfrb_classifier_load": ([vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
            "nsfrb_classifier_activations_get": ([vp, i32, i32, vp], ctypes.c_int),
            "nsfrb_classifier_grad_pre_get": ([vp, i32, i32, vp], ctypes.c_int),
            "nsfrb_classifier_logits_get": ([vp, i32, pf], ctypes.c_int),
            "nsfrb_inject_rfi": ([vp, i32, i32, i32, i32, i32, i32, i32, i32, i32, ctypes.c_float, vp], ctypes.c_int),
            "nsfrb_classifier_param_count": ([], ctypes.c_int32),
            "nsfrb_classifier_create": ([ctypes.POINTER(ClassifierConfig), ctypes.POINTER(vp)], ctypes.c_int),
            "nsfrb_classifier_destroy": ([vp], ctypes.c_int),
            "nsfrb_classifier_params_get": ([vp, pf], ctypes.c_int),
            "nsfrb_classifier_params_set": ([vp, pf], ctypes.c_int),
            "nsfrb_classifier_grads_get": ([vp, pf], ctypes.c_int),
            "nsfrb_classifier_set_lr": ([vp, ctypes.c_float], ctypes.c_int),
            "nsfrb_classifier_train_step": ([vp, vp, vp, i32, i32, pf, vp], ctypes.c_int),
            "nsfrb_classifier_infer": ([vp, vp, i32, vp, vp], ctypes.c_int),
            "nsfrb_cutouts_extract": ([vp, ctypes.POINTER(vp), i32, i32, i32, i32, i32, i32, pi32, i32,
                                       ctypes.POINTER(CutoutDesc), i32, vp, vp], ctypes.c_int),
            "nsfrb_bin_time": ([vp, i32, i32, i32, i32, i32, vp, vp], ctypes.c_int),
            "nsfrb_plan_dm_grid": ([ctypes.c_double] * 8 + [pd, i32, pi32], ctypes.c_int),
            "nsfrb_psf_reduce": ([ctypes.POINTER(Candidate), i32, pf, i32, i32, ctypes.c_double, pi32, pd],
                                 ctypes.c_int),
            "nsfrb_stream_create": ([ctypes.POINTER(Config), i32, ctypes.c_double, ctypes.POINTER(vp)], ctypes.c_int),
            "nsfrb_stream_destroy": ([vp], ctypes.c_int),
            "nsfrb_stream_push": ([vp, vp, vp, ctypes.POINTER(StreamResult)], ctypes.c_int),
            "nsfrb_stream_search": ([vp, ctypes.POINTER(vp)], ctypes.c_int),
            "nsfrb_multiscale_create": ([ctypes.POINTER(Config), i32, pi32, pd, ctypes.POINTER(vp)], ctypes.c_int),
            "nsfrb_multiscale_destroy": ([vp], ctypes.c_int),
            "nsfrb_multiscale_run": ([vp, vp, vp], ctypes.c_int),
            "nsfrb_multiscale_scale": ([vp, i32, ctypes.POINTER(vp)], ctypes.c_int),
            "nsfrb_multiscale_candidates_get": ([vp, ctypes.POINTER(ScaleCandidate), i32, pi32, pi32],
                                                ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes, f.restype = args, res
        _lib = L
    return _lib


def last_error():
    return lib().nsfrb_last_error().decode()


def check(status):
    if status != OK:
        raise NsfrbError(status, last_error())
    return status


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class SearchConfig:
    """Owns the host arrays behind a C `nsfrb_search_config`."""

    def __init__(self, nx, ny, n_time, freqs_ghz, dms, widths, f_ref_ghz=None, dt_ms=134.2,
                 k_dm_ms=4.15, in_dtype="f32", store_dtype="f32", norm="pixel_subband",
                 snr_threshold=6.0, max_candidates=10, device=0, layout="tsp"):
        self.freqs = np.ascontiguousarray(freqs_ghz, dtype=np.float64)
        self.dms = np.ascontiguousarray(dms, dtype=np.float64)
        self.widths = np.ascontiguousarray(widths, dtype=np.int32)
        self.nx, self.ny, self.n_time = int(nx), int(ny), int(n_time)
        self.n_sub = int(self.freqs.size)
        self.in_dtype, self.store_dtype, self.norm, self.layout = in_dtype, store_dtype, norm, layout
        self.max_candidates = int(max_candidates)
        c = Config()
        c.struct_size = ctypes.sizeof(Config)
        c.nx, c.ny, c.n_sub, c.n_time = self.nx, self.ny, self.n_sub, self.n_time
        c.freq_ghz = _ptr(self.freqs, ctypes.c_double)
        c.f_ref_ghz = float(self.freqs.max() if f_ref_ghz is None else f_ref_ghz)
        c.dt_ms, c.k_dm_ms = float(dt_ms), float(k_dm_ms)
        c.n_dm, c.dm = int(self.dms.size), _ptr(self.dms, ctypes.c_double)
        c.n_width, c.width = int(self.widths.size), _ptr(self.widths, ctypes.c_int32)
        c.in_dtype, c.store_dtype, c.norm = DTYPES[in_dtype], DTYPES[store_dtype], NORMS[norm]
        c.snr_threshold = float(snr_threshold)
        c.max_candidates = self.max_candidates
        c.device = int(device)
        c.layout = LAYOUTS[layout]
        self.c = c

    @property
    def n_pix(self):
        return self.nx * self.ny

    def derived(self, n_time, dt_ms, dms, in_dtype):
        """The same search with another time axis, DM list and input dtype."""
        c = self.c
        return SearchConfig(self.nx, self.ny, n_time, self.freqs, dms, self.widths, f_ref_ghz=c.f_ref_ghz,
                            dt_ms=dt_ms, k_dm_ms=c.k_dm_ms, in_dtype=in_dtype, store_dtype=self.store_dtype,
                            norm=self.norm, snr_threshold=c.snr_threshold, max_candidates=self.max_candidates,
                            device=c.device, layout=self.layout)

    def validate(self):
        return lib().nsfrb_config_validate(ctypes.byref(self.c))

    def delays(self):
        out = np.zeros((self.dms.size, self.n_sub), dtype=np.int32)
        check(lib().nsfrb_plan_delays(ctypes.byref(self.c), _ptr(out, ctypes.c_int32)))
        return out

    def plan_source(self, compile=False):
        n = lib().nsfrb_debug_plan_source(ctypes.byref(self.c), None, 0, 0)
        if n < 0:
            raise NsfrbError(INVALID_ARG, last_error())
        buf = ctypes.create_string_buffer(n + 1)
        r = lib().nsfrb_debug_plan_source(ctypes.byref(self.c), buf, n + 1, 1 if compile else 0)
        if r < 0:
            raise NsfrbError(DEVICE, last_error())
        return buf.value.decode()


def plan_dm_grid(nu_min_ghz, nu_max_ghz, chan_bw_mhz, t_s_ms, w_int_ms, tol, dm_min, dm_max):
    """nsfrb_plan_dm_grid: DM trials from a smearing tolerance (host only)."""
    n = ctypes.c_int32()
    args = [float(v) for v in (nu_min_ghz, nu_max_ghz, chan_bw_mhz, t_s_ms, w_int_ms, tol, dm_min, dm_max)]
    st = lib().nsfrb_plan_dm_grid(*args, None, 0, ctypes.byref(n))
    if st not in (OK, TRUNCATED):
        check(st)
    out = np.zeros(n.value, np.float64)
    check(lib().nsfrb_plan_dm_grid(*args, _ptr(out, ctypes.c_double), n.value, ctypes.byref(n)))
    return out


def psf_reduce(cands, psf, percentile=90.0):
    """nsfrb_psf_reduce: index of the most likely candidate and its weighted mean S/N.
    cands: dicts with x, y, snr (e.g. from Search.candidates) in list order."""
    arr = (Candidate * len(cands))()
    for i, c in enumerate(cands):
        arr[i].x, arr[i].y, arr[i].snr = int(c["x"]), int(c["y"]), float(c["snr"])
        arr[i].dm_index, arr[i].width_index, arr[i].toa = int(c.get("dm_index", 0)), int(c.get("width_index", 0)), \
            int(c.get("toa", 0))
    p = np.ascontiguousarray(psf, dtype=np.float32)
    idx, score = ctypes.c_int32(), ctypes.c_double()
    check(lib().nsfrb_psf_reduce(arr, len(cands), _ptr(p, ctypes.c_float), p.shape[1], p.shape[0], float(percentile),
                                 ctypes.byref(idx), ctypes.byref(score)))
    return idx.value, score.value


def bin_time(d_x, in_dtype, n_time, n_sub, n_pix, factor, d_out, stream=0):
    """nsfrb_bin_time: FP32 [n_time // factor][n_sub][n_pix] sums of consecutive samples."""
    check(lib().nsfrb_bin_time(ctypes.c_void_p(int(d_x)), DTYPES[in_dtype], int(n_time), int(n_sub), int(n_pix),
                               int(factor), ctypes.c_void_p(int(d_out)), ctypes.c_void_p(int(stream))))


class MultiScale:
    """Searches of one raw cube at several timescales (nsfrb_multiscale_*).

    Timescale s bins by factors[s] and searches with dt * factors[s] and the DM
    trials times dm_scales[s] (0: DM 0 only). The default is the paper's three
    timescales: native, 5x binned at 5x the DMs, 75x binned without
    de-dispersion."""

    def __init__(self, cfg: SearchConfig, factors=(1, 5, 75), dm_scales=(1.0, 5.0, 0.0)):
        self.factors = [int(f) for f in factors]
        self.dm_scales = [float(d) for d in dm_scales]
        n = len(self.factors)
        f_arr = (ctypes.c_int32 * n)(*self.factors)
        d_arr = (ctypes.c_double * n)(*self.dm_scales)
        h = ctypes.c_void_p()
        check(lib().nsfrb_multiscale_create(ctypes.byref(cfg.c), n, f_arr, d_arr, ctypes.byref(h)))
        self.h, self.cfg = h, cfg
        self.cfgs = []
        for f, k in zip(self.factors, self.dm_scales):
            dms = cfg.dms * k if k != 0.0 else np.zeros(1)
            self.cfgs.append(cfg.derived(cfg.n_time // f, cfg.c.dt_ms * f, dms, cfg.in_dtype if f == 1 else "f32"))

    def close(self):
        if getattr(self, "h", None):
            lib().nsfrb_multiscale_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def run(self, d_cube_ptr, stream=0):
        check(lib().nsfrb_multiscale_run(self.h, ctypes.c_void_p(int(d_cube_ptr)), ctypes.c_void_p(int(stream))))

    def scale(self, s):
        """Search view of timescale s (maps, best, noise statistics, z cube...)."""
        p = ctypes.c_void_p()
        check(lib().nsfrb_multiscale_scale(self.h, int(s), ctypes.byref(p)))
        return Search._borrow(self.cfgs[s], p, self)

    def candidates(self, capacity=None):
        cap = self.cfg.max_candidates if capacity is None else int(capacity)
        arr = (ScaleCandidate * max(cap, 1))()
        nw, nt = ctypes.c_int32(), ctypes.c_int32()
        st = lib().nsfrb_multiscale_candidates_get(self.h, arr, cap, ctypes.byref(nw), ctypes.byref(nt))
        if st not in (OK, TRUNCATED):
            check(st)
        recs = [dict(x=r.cand.x, y=r.cand.y, dm_index=r.cand.dm_index, width_index=r.cand.width_index,
                     toa=r.cand.toa, snr=r.cand.snr, scale=r.scale) for r in arr[:nw.value]]
        return recs, nt.value, st


class Stream:
    """Real-time form (nsfrb_stream_*): batches of `chunk` samples into a ring of
    cfg.n_time samples, the window searched after each batch once full."""

    def __init__(self, cfg: SearchConfig, chunk=25, deadline_ms=3350.0):
        h = ctypes.c_void_p()
        check(lib().nsfrb_stream_create(ctypes.byref(cfg.c), int(chunk), float(deadline_ms), ctypes.byref(h)))
        self.h, self.cfg, self.chunk = h, cfg, int(chunk)

    def close(self):
        if getattr(self, "h", None):
            lib().nsfrb_stream_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def push(self, d_chunk_ptr, stream=0):
        r = StreamResult()
        check(lib().nsfrb_stream_push(self.h, ctypes.c_void_p(int(d_chunk_ptr)), ctypes.c_void_p(int(stream)),
                                      ctypes.byref(r)))
        c = r.cand
        return dict(searched=bool(r.searched), has_candidate=bool(r.has_candidate), chunk_index=r.chunk_index,
                    window_start=r.window_start, search_ms=r.search_ms, dropped_total=r.dropped_total,
                    flagged=r.flagged,
                    cand=dict(x=c.x, y=c.y, dm_index=c.dm_index, width_index=c.width_index, toa=c.toa, snr=c.snr)
                    if r.has_candidate else None)

    def search(self):
        """Search view of the last searched window (maps, statistics, z cube)."""
        p = ctypes.c_void_p()
        check(lib().nsfrb_stream_search(self.h, ctypes.byref(p)))
        return Search._borrow(self.cfg, p, self)


class Search:
    """A search plan on one GPU (nsfrb_search_create / run / candidates_get)."""

    def __init__(self, cfg: SearchConfig):
        self.cfg = cfg
        h = ctypes.c_void_p()
        check(lib().nsfrb_search_create(ctypes.byref(cfg.c), ctypes.byref(h)))
        self.h = h

    @classmethod
    def _borrow(cls, cfg, handle, owner):
        """A view of a search handle owned by another object (not destroyed here)."""
        obj = cls.__new__(cls)
        obj.cfg, obj.h, obj._owner = cfg, handle, owner
        return obj

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self.h = None
            return
        if getattr(self, "h", None):
            lib().nsfrb_search_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def run(self, d_cube_ptr, stream=0):
        check(lib().nsfrb_search_run(self.h, ctypes.c_void_p(int(d_cube_ptr)), ctypes.c_void_p(int(stream))))

    def candidates(self, capacity=None):
        cap = self.cfg.max_candidates if capacity is None else int(capacity)
        arr = (Candidate * max(cap, 1))()
        nw, nt = ctypes.c_int32(), ctypes.c_int32()
        st = lib().nsfrb_candidates_get(self.h, arr, cap, ctypes.byref(nw), ctypes.byref(nt))
        if st not in (OK, TRUNCATED):
            check(st)
        recs = [dict(x=c.x, y=c.y, dm_index=c.dm_index, width_index=c.width_index, toa=c.toa, snr=c.snr)
                for c in arr[:nw.value]]
        return recs, nt.value, st

    def maps(self):
        c = self.cfg
        shape = (c.dms.size, c.widths.size, c.n_pix)
        snr = np.zeros(shape, np.float32)
        toa = np.zeros(shape, np.int32)
        check(lib().nsfrb_maps_get(self.h, _ptr(snr, ctypes.c_float), _ptr(toa, ctypes.c_int32)))
        return snr, toa

    def best(self):
        n = self.cfg.n_pix
        s = np.zeros(n, np.float32)
        d, w, t = (np.zeros(n, np.int32) for _ in range(3))
        check(lib().nsfrb_best_get(self.h, _ptr(s, ctypes.c_float), _ptr(d, ctypes.c_int32),
                                   _ptr(w, ctypes.c_int32), _ptr(t, ctypes.c_int32)))
        return s, d, w, t

    def noise_stats(self):
        n = (self.cfg.n_pix, self.cfg.n_sub)
        med, sig = np.zeros(n), np.zeros(n)
        check(lib().nsfrb_noise_stats_get(self.h, _ptr(med, ctypes.c_double), _ptr(sig, ctypes.c_double)))
        return med, sig

    def set_noise_stats(self, med, sigma):
        med = np.ascontiguousarray(med, dtype=np.float64)
        sig = np.ascontiguousarray(sigma, dtype=np.float64)
        check(lib().nsfrb_noise_stats_set(self.h, _ptr(med, ctypes.c_double), _ptr(sig, ctypes.c_double)))

    def zcube(self):
        """Normalised cube [p][s][t] as float64 values of the store dtype."""
        c = self.cfg
        n = c.n_pix * c.n_sub * c.n_time
        if c.store_dtype == "f32":
            raw = np.zeros(n, np.float32)
        else:
            raw = np.zeros(n, np.uint16)
        check(lib().nsfrb_zcube_get(self.h, raw.ctypes.data_as(ctypes.c_void_p)))
        if c.store_dtype == "f16":
            vals = raw.view(np.float16).astype(np.float64)
        elif c.store_dtype == "bf16":
            vals = (raw.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        else:
            vals = raw.astype(np.float64)
        return vals.reshape(c.n_pix, c.n_sub, c.n_time), raw.reshape(c.n_pix, c.n_sub, c.n_time)

    def zcube_device(self):
        """Device address of the normalised cube of the last run (no wait)."""
        p = ctypes.c_void_p()
        check(lib().nsfrb_zcube_device(self.h, ctypes.byref(p)))
        return int(p.value)

    def flag_count(self):
        v = ctypes.c_int64()
        check(lib().nsfrb_flag_count_get(self.h, ctypes.byref(v)))
        return v.value

    def profiling(self, on=True):
        check(lib().nsfrb_profiling_enable(self.h, 1 if on else 0))

    def stage_times_ms(self):
        out = np.zeros(3, np.float32)
        check(lib().nsfrb_stage_times_get(self.h, _ptr(out, ctypes.c_float)))
        return out

    def delay_table(self):
        out = np.zeros((self.cfg.dms.size, self.cfg.n_sub), np.int32)
        check(lib().nsfrb_delay_table_get(self.h, _ptr(out, ctypes.c_int32)))
        return out

    def plan_info(self):
        out = np.zeros(9, np.int32)
        check(lib().nsfrb_search_plan_info(self.h, _ptr(out, ctypes.c_int32)))
        return dict(samples_per_lane=int(out[0]), pixels_per_workgroup=int(out[1]), row_len=int(out[2]),
                    lds_bytes=int(out[3]), threads_per_workgroup=int(out[4]), persistent=bool(out[5]),
                    lds_buffers=int(out[6]), workgroups=int(out[7]))


class Batch:
    """Many uneven cubes searched by one persistent, graph-captured launch."""

    def __init__(self, cfgs):
        self.cfgs = list(cfgs)
        arr = (Config * len(self.cfgs))(*[c.c for c in self.cfgs])
        self._arr = arr
        h = ctypes.c_void_p()
        check(lib().nsfrb_batch_create(arr, len(self.cfgs), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().nsfrb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _ptrs(self, ptrs):
        return (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(int(p)) for p in ptrs])

    def run(self, ptrs, stream=0):
        check(lib().nsfrb_batch_run(self.h, self._ptrs(ptrs), ctypes.c_void_p(int(stream))))

    def run_separate(self, ptrs, stream=0):
        check(lib().nsfrb_batch_run_separate(self.h, self._ptrs(ptrs), ctypes.c_void_p(int(stream))))

    def use_graph(self, on=True):
        check(lib().nsfrb_batch_use_graph(self.h, 1 if on else 0))

    def candidates(self, i):
        cap = self.cfgs[i].max_candidates
        arr = (Candidate * cap)()
        nw, nt = ctypes.c_int32(), ctypes.c_int32()
        st = lib().nsfrb_batch_candidates_get(self.h, i, arr, cap, ctypes.byref(nw), ctypes.byref(nt))
        if st not in (OK, TRUNCATED):
            check(st)
        return [dict(x=c.x, y=c.y, dm_index=c.dm_index, width_index=c.width_index, toa=c.toa, snr=c.snr)
                for c in arr[:nw.value]], nt.value

    def maps(self, i):
        c = self.cfgs[i]
        shape = (c.dms.size, c.widths.size, c.n_pix)
        snr = np.zeros(shape, np.float32)
        toa = np.zeros(shape, np.int32)
        check(lib().nsfrb_batch_maps_get(self.h, i, _ptr(snr, ctypes.c_float), _ptr(toa, ctypes.c_int32)))
        return snr, toa

    def best(self, i):
        n = self.cfgs[i].n_pix
        s = np.zeros(n, np.float32)
        d, w, t = (np.zeros(n, np.int32) for _ in range(3))
        check(lib().nsfrb_batch_best_get(self.h, i, _ptr(s, ctypes.c_float), _ptr(d, ctypes.c_int32),
                                         _ptr(w, ctypes.c_int32), _ptr(t, ctypes.c_int32)))
        return s, d, w, t

    def zcube_device(self, i):
        p = ctypes.c_void_p()
        check(lib().nsfrb_batch_zcube_device(self.h, i, ctypes.byref(p)))
        return int(p.value)

    def info(self):
        out = np.zeros(5, np.int64)
        check(lib().nsfrb_batch_info_get(self.h, _ptr(out, ctypes.c_int64)))
        return dict(work_items=int(out[0]), grid=int(out[1]), lds_bytes=int(out[2]), classes=int(out[3]),
                    graph=bool(out[4]))


def generate_noise(d_ptr, dtype, layout, n_pix, n_sub, n_time, seed, sigma=1.0, stream=0):
    check(lib().nsfrb_generate_noise(ctypes.c_void_p(int(d_ptr)), DTYPES[dtype], LAYOUTS[layout], n_pix, n_sub,
                                     n_time, ctypes.c_uint64(seed), float(sigma), ctypes.c_void_p(int(stream))))


def inject_boxcar(d_ptr, dtype, layout, n_pix, n_sub, n_time, pixel, t0, width, amp, offsets, stream=0):
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    assert off.size == n_sub
    check(lib().nsfrb_inject_boxcar(ctypes.c_void_p(int(d_ptr)), DTYPES[dtype], LAYOUTS[layout], n_pix, n_sub,
                                    n_time, int(pixel), int(t0), int(width), float(amp), _ptr(off, ctypes.c_int32),
                                    ctypes.c_void_p(int(stream))))


def inject_boxcars(d_ptrs, dtype, layout, n_pix, n_sub, n_time, boxcars, offsets, stream=0, static=False):
    """boxcars: (cube, pixel, t0, width, amp) tuples; offsets: [n][n_sub] sample shifts.

    static=True calls nsfrb_inject_boxcars_static (tables staged in the
    library's static device array; no device allocation)."""
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    n = len(boxcars)
    assert off.shape == (n, n_sub)
    ptrs = (ctypes.c_void_p * len(d_ptrs))(*[ctypes.c_void_p(int(p)) for p in d_ptrs])
    recs = (Boxcar * n)(*[Boxcar(int(k), int(p), int(t), int(w), float(a)) for (k, p, t, w, a) in boxcars])
    fn = lib().nsfrb_inject_boxcars_static if static else lib().nsfrb_inject_boxcars
    check(fn(ptrs, len(d_ptrs), DTYPES[dtype], LAYOUTS[layout], n_pix, n_sub, n_time, recs,
             _ptr(off, ctypes.c_int32), n, ctypes.c_void_p(int(stream))))


def philox_fill(d_ptr, n_blocks, seed, stream=0):
    check(lib().nsfrb_philox_fill(ctypes.c_void_p(int(d_ptr)), int(n_blocks), ctypes.c_uint64(seed),
                                  ctypes.c_void_p(int(stream))))


def inject_rfi(d_ptr, dtype, layout, n_pix, n_sub, n_time, kind, t0, length=1, sub_band=0, amp=1.0, stream=0):
    """kind 'spike': one sample, all sub-bands; kind 'stripe': one sub-band over [t0, t0+length)."""
    k = {"spike": 0, "stripe": 1}[kind]
    check(lib().nsfrb_inject_rfi(ctypes.c_void_p(int(d_ptr)), DTYPES[dtype], LAYOUTS[layout], n_pix, n_sub, n_time,
                                 k, int(t0), int(length), int(sub_band), float(amp), ctypes.c_void_p(int(stream))))


class Classifier:
    """The candidate classifier (3-D CNN, BF16 MFMA training and inference)."""

    def __init__(self, max_batch=64, n_time=64, ny=32, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=1,
                 device=0):
        c = ClassifierConfig()
        c.struct_size = ctypes.sizeof(ClassifierConfig)
        c.max_batch, c.n_time, c.ny = int(max_batch), int(n_time), int(ny)
        c.lr, c.beta1, c.beta2, c.eps = float(lr), float(beta1), float(beta2), float(eps)
        c.seed, c.device = int(seed), int(device)
        self.cfg = c
        h = ctypes.c_void_p()
        check(lib().nsfrb_classifier_create(ctypes.byref(c), ctypes.byref(h)))
        self.h = h
        self.n_params = int(lib().nsfrb_classifier_param_count())

    def close(self):
        if getattr(self, "h", None):
            lib().nsfrb_classifier_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def params(self):
        out = np.zeros(self.n_params, np.float32)
        check(lib().nsfrb_classifier_params_get(self.h, _ptr(out, ctypes.c_float)))
        return out

    def set_params(self, theta):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        assert t.size == self.n_params
        check(lib().nsfrb_classifier_params_set(self.h, _ptr(t, ctypes.c_float)))

    def set_lr(self, lr):
        check(lib().nsfrb_classifier_set_lr(self.h, float(lr)))

    def grads(self):
        out = np.zeros(self.n_params, np.float32)
        check(lib().nsfrb_classifier_grads_get(self.h, _ptr(out, ctypes.c_float)))
        return out

    def activations(self, layer, n):
        """BF16 output of conv layer 1..4 from the last forward pass, as float32 [n][T][Y][32][32]."""
        c = self.cfg
        bits = np.zeros(n * c.n_time * c.ny * 32 * 32, np.uint16)
        check(lib().nsfrb_classifier_activations_get(self.h, int(layer), int(n), _ptr(bits, ctypes.c_uint16)))
        return (bits.astype(np.uint32) << 16).view(np.float32).reshape(n, c.n_time, c.ny, 32, 32)

    def grad_pre(self, layer, n):
        """BF16 gradient at conv layer 1..4's pre-activation from the last train step, float32 [n][T][Y][32][32]."""
        c = self.cfg
        bits = np.zeros(n * c.n_time * c.ny * 32 * 32, np.uint16)
        check(lib().nsfrb_classifier_grad_pre_get(self.h, int(layer), int(n), _ptr(bits, ctypes.c_uint16)))
        return (bits.astype(np.uint32) << 16).view(np.float32).reshape(n, c.n_time, c.ny, 32, 32)

    def logits(self, n):
        out = np.zeros(n, np.float32)
        check(lib().nsfrb_classifier_logits_get(self.h, int(n), _ptr(out, ctypes.c_float)))
        return out

    def state(self, user_counter=0):
        """Checkpoint bytes: weights, Adam moments, step count, optimiser settings, user_counter."""
        n = int(lib().nsfrb_classifier_state_bytes())
        buf = np.zeros(n, np.uint8)
        written = ctypes.c_int64(0)
        check(lib().nsfrb_classifier_save(self.h, ctypes.c_uint64(int(user_counter)), _ptr(buf, ctypes.c_uint8), n,
                                          ctypes.byref(written)))
        return buf.tobytes()

    def load_state(self, blob):
        """Restore a checkpoint from state(); returns its user_counter."""
        b = np.frombuffer(bytes(blob), np.uint8)
        ctr = ctypes.c_uint64(0)
        check(lib().nsfrb_classifier_load(self.h, _ptr(b, ctypes.c_uint8), b.size, ctypes.byref(ctr)))
        return int(ctr.value)

    def save(self, path, user_counter=0):
        with open(path, "wb") as f:
            f.write(self.state(user_counter))

    def load(self, path):
        with open(path, "rb") as f:
            return self.load_state(f.read())

    def train_step(self, d_cutouts, d_labels, n, update=True, stream=0, want_loss=True):
        loss = ctypes.c_float(float("nan"))
        check(lib().nsfrb_classifier_train_step(self.h, ctypes.c_void_p(int(d_cutouts)), ctypes.c_void_p(int(d_labels)),
                                                int(n), 1 if update else 0,
                                                ctypes.byref(loss) if want_loss else None,
                                                ctypes.c_void_p(int(stream))))
        return loss.value

    def infer(self, d_cutouts, n, d_prob, stream=0):
        check(lib().nsfrb_classifier_infer(self.h, ctypes.c_void_p(int(d_cutouts)), int(n),
                                           ctypes.c_void_p(int(d_prob)), ctypes.c_void_p(int(stream))))

    def cutouts(self, d_z_cubes, store_dtype, nx, ny, n_sub, n_time, delays, descs, d_out, stream=0):
        """d_z_cubes: device addresses of the cubes; descs: (cube, px, py, dm_index, toa) tuples."""
        dl = np.ascontiguousarray(delays, dtype=np.int32)
        ptrs = (ctypes.c_void_p * len(d_z_cubes))(*[ctypes.c_void_p(int(p)) for p in d_z_cubes])
        arr = (CutoutDesc * len(descs))(*[CutoutDesc(int(k), int(x), int(y), int(d), int(t))
                                            for (k, x, y, d, t) in descs])
        check(lib().nsfrb_cutouts_extract(self.h, ptrs, len(d_z_cubes), DTYPES[store_dtype], int(nx), int(ny),
                                          int(n_sub), int(n_time), _ptr(dl, ctypes.c_int32), dl.shape[0],
                                          arr, len(descs), ctypes.c_void_p(int(d_out)), ctypes.c_void_p(int(stream))))
