"""ctypes binding of libndconv.so: the C ABI of include/ndconv.h with the
same names and argument order.  Marshalling only; every step of the
computation runs in the library's HIP kernels.  Importing this module fails
loudly when the library has not been built."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libndconv.so")

NDC_OK, NDC_EINVAL, NDC_EUNSUPPORTED, NDC_EALIAS = 0, -1, -2, -3
NDC_ENONFINITE, NDC_EDEVICE, NDC_EWORKSPACE = -4, -5, -6
NDC_F32, NDC_F64 = 0, 1
NDC_PREC_NATIVE, NDC_PREC_BF16, NDC_PREC_SPLIT_BF16 = 0, 1, 2
NDC_STOP_DONE, NDC_STOP_NO_DESCENT, NDC_STOP_TRIALS = 0, 1, 2
NDC_MAX_ITERS = 1 << 24

NDC_DH_SCRATCH_BYTES = 1 << 25

EXPORTS = ("conv_full_nd", "conv_adjoint_nd", "conv_dH_workspace_bytes", "conv_dH_nd", "conv_dH_nd_noalloc",
           "deconv_workspace_bytes", "deconv_iterate", "deconv_workspace_bytes_ex", "deconv_iterate_ex",
           "rl_workspace_bytes", "rl_iterate", "ndc_batch_plan_create", "ndc_batch_plan_destroy",
           "ndc_batch_workspace_bytes", "ndc_batch_plan_info", "ndc_batch_conv_full", "ndc_batch_conv_adjoint",
           "ndc_batch_deconv", "ndc_tile_override", "ndc_tile_override_clear", "ndc_tile_choice", "ndc_strerror",
           "ndc_version")
NDC_FORM_AUTO, NDC_FORM_VALU, NDC_FORM_SMALL, NDC_FORM_MFMA4, NDC_FORM_MFMA32, NDC_FORM_SLOT = 0, 1, 2, 3, 4, 5


class NdcError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (what or "ndconv", strerror(status), status))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libndconv.so is not built; run __graft_entry__.build() or "
                          "python paper_1711_11224_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    i64p = ctypes.POINTER(ctypes.c_int64)
    vp, c_int, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    lib.conv_full_nd.argtypes = [c_int, i64p, i64p, vp, vp, vp, c_int, c_int, vp]
    lib.conv_full_nd.restype = c_int
    lib.conv_adjoint_nd.argtypes = [c_int, i64p, i64p, vp, vp, vp, c_int, c_int, vp]
    lib.conv_adjoint_nd.restype = c_int
    lib.conv_dH_workspace_bytes.argtypes = [c_int, i64p, i64p, c_int]
    lib.conv_dH_workspace_bytes.restype = sz
    lib.conv_dH_nd.argtypes = [c_int, i64p, i64p, vp, vp, vp, c_int, vp, sz, vp]
    lib.conv_dH_nd.restype = c_int
    lib.conv_dH_nd_noalloc.argtypes = [c_int, i64p, i64p, vp, vp, vp, c_int, vp]
    lib.conv_dH_nd_noalloc.restype = c_int
    lib.deconv_workspace_bytes.argtypes = [c_int, i64p, i64p, c_int, c_int]
    lib.deconv_workspace_bytes.restype = sz
    lib.deconv_iterate.argtypes = [c_int, i64p, i64p, vp, vp, vp, c_int, ctypes.c_double, c_int, c_int,
                                   vp, sz, vp, vp, vp]
    lib.deconv_iterate.restype = c_int
    lib.deconv_workspace_bytes_ex.argtypes = [c_int, i64p, i64p, c_int, c_int, c_int]
    lib.deconv_workspace_bytes_ex.restype = sz
    lib.deconv_iterate_ex.argtypes = [c_int, i64p, i64p, vp, vp, vp, c_int, ctypes.c_double, ctypes.c_double, c_int,
                                      c_int, c_int, c_int, vp, sz, vp, vp, vp]
    lib.deconv_iterate_ex.restype = c_int
    lib.rl_workspace_bytes.argtypes = [c_int, i64p, i64p, c_int, c_int]
    lib.rl_workspace_bytes.restype = sz
    lib.rl_iterate.argtypes = [c_int, i64p, i64p, vp, vp, vp, c_int, c_int, c_int, vp, sz, vp, vp, vp]
    lib.rl_iterate.restype = c_int
    pvp = ctypes.POINTER(ctypes.c_void_p)
    lib.ndc_batch_plan_create.argtypes = [c_int, i64p, i64p, c_int, c_int, ctypes.POINTER(c_int), pvp]
    lib.ndc_batch_plan_create.restype = c_int
    lib.ndc_batch_plan_destroy.argtypes = [vp]
    lib.ndc_batch_plan_destroy.restype = None
    lib.ndc_batch_workspace_bytes.argtypes = [vp]
    lib.ndc_batch_workspace_bytes.restype = sz
    lib.ndc_batch_plan_info.argtypes = [vp, i64p]
    lib.ndc_batch_plan_info.restype = c_int
    lib.ndc_batch_conv_full.argtypes = [vp, pvp, pvp, pvp, vp]
    lib.ndc_batch_conv_full.restype = c_int
    lib.ndc_batch_conv_adjoint.argtypes = [vp, pvp, pvp, pvp, vp]
    lib.ndc_batch_conv_adjoint.restype = c_int
    lib.ndc_batch_deconv.argtypes = [vp, pvp, pvp, pvp, c_int, ctypes.c_double, vp, sz, pvp, vp, vp]
    lib.ndc_batch_deconv.restype = c_int
    lib.ndc_tile_override.argtypes = [c_int, i64p, i64p, c_int, c_int, c_int, c_int, c_int]
    lib.ndc_tile_override.restype = c_int
    lib.ndc_tile_override_clear.argtypes = []
    lib.ndc_tile_override_clear.restype = None
    lib.ndc_tile_choice.argtypes = [c_int, i64p, i64p, c_int, c_int, c_int, ctypes.POINTER(c_int)]
    lib.ndc_tile_choice.restype = c_int
    lib.ndc_strerror.argtypes = [c_int]
    lib.ndc_strerror.restype = ctypes.c_char_p
    lib.ndc_version.argtypes = []
    lib.ndc_version.restype = c_int
    return lib


lib = _load()


def strerror(status: int) -> str:
    return lib.ndc_strerror(int(status)).decode()


def i64_array(vals):
    arr = (ctypes.c_int64 * max(1, len(vals)))(*[int(v) for v in vals])
    return arr


def check(status, what):
    if status != NDC_OK:
        raise NdcError(status, what)
