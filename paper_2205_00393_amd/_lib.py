"""ctypes declarations of libltn (see include/ltn.h). Marshalling only."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libltn.so")

LTN_OK = 0
LTN_C64, LTN_SPLIT_F16, LTN_SPLIT_BF16 = 0, 1, 2
MODES = {"c64": LTN_C64, "split_f16": LTN_SPLIT_F16, "split_bf16": LTN_SPLIT_BF16}
LTN_GATE_SQRT_X, LTN_GATE_SQRT_Y, LTN_GATE_SQRT_W, LTN_GATE_FSIM, LTN_GATE_U3, LTN_GATE_MATRIX = 1, 2, 3, 4, 5, 6
LTN_K_SMALL, LTN_K_MFMA = 0, 1


class LtnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ltn error {code}: {msg}")
        self.code = code


class Gate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32), ("param_id", C.c_int32),
                ("p", C.c_double * 3), ("m", C.c_double * 32)]


class Network(C.Structure):
    _fields_ = [("n_leaves", C.c_int32), ("leaf_off", C.POINTER(C.c_int64)),
                ("index_ids", C.POINTER(C.c_int32)), ("leaf_data", C.POINTER(C.c_float)),
                ("n_open", C.c_int32), ("open_ids", C.POINTER(C.c_int32)),
                ("n_indices", C.c_int32), ("param_leaf", C.POINTER(C.c_int32))]


class Costs(C.Structure):
    _fields_ = [("log2_cost", C.c_double), ("log2_sliced", C.c_double), ("overhead", C.c_double),
                ("space_log2", C.c_int32), ("space_log2_unsliced", C.c_int32),
                ("cost_words", C.c_uint64 * 4), ("sliced_words", C.c_uint64 * 4),
                ("stem_len", C.c_int32)]


class StemRow(C.Structure):
    _fields_ = [("tensor", C.c_int32), ("rank", C.c_int32), ("rank_sliced", C.c_int32),
                ("node_bits", C.c_int32), ("node_bits_sliced", C.c_int32)]


class SearchOpts(C.Structure):
    _fields_ = [("n_alpha", C.c_int32), ("alphas", C.POINTER(C.c_double)),
                ("n_tau", C.c_int32), ("taus", C.POINTER(C.c_double)),
                ("n_seeds", C.c_int32), ("seed_base", C.c_uint64), ("reconf_k", C.c_int32),
                ("reconf_sweeps", C.c_int32)]


class RefineOpts(C.Structure):
    _fields_ = [("t0", C.c_double), ("alpha", C.c_double), ("tf", C.c_double),
                ("iters_per_temp", C.c_int32), ("n_fixed", C.c_int32), ("seed", C.c_uint64)]


class RefineStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("proposals", C.c_int32), ("accepted", C.c_int32),
                ("dropped", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("max_rank", C.c_int32), ("batch", C.c_int32), ("fat_threshold", C.c_int32),
                ("fuse_rank", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("n_leaves", C.c_int32), ("n_steps", C.c_int32), ("n_sliced", C.c_int32),
                ("n_open", C.c_int32), ("n_open_unsliced", C.c_int32), ("n_params", C.c_int32),
                ("batch", C.c_int32), ("root_rank", C.c_int32), ("macs_per_slice", C.c_double),
                ("macs_words", C.c_uint64 * 2), ("arena_bytes_per_slice", C.c_uint64),
                ("grad_arena_bytes_per_slice", C.c_uint64), ("const_bytes", C.c_uint64),
                ("sliced_ids", C.POINTER(C.c_int32))]


class StepInfo(C.Structure):
    _fields_ = [("left", C.c_int32), ("right", C.c_int32), ("out", C.c_int32),
                ("a_is_left", C.c_int32), ("m", C.c_int32), ("k", C.c_int32), ("n", C.c_int32),
                ("kernel", C.c_int32), ("a_idx", C.POINTER(C.c_int32)),
                ("b_idx", C.POINTER(C.c_int32)), ("c_idx", C.POINTER(C.c_int32)),
                ("c_mask_a", C.c_uint64), ("arena_off_a", C.c_uint64),
                ("arena_off_b", C.c_uint64), ("arena_off_c", C.c_uint64)]


P = C.c_void_p
I32, U64, D = C.c_int32, C.c_uint64, C.c_double
I32P, U64P, DP = C.POINTER(C.c_int32), C.POINTER(C.c_uint64), C.POINTER(C.c_double)

SIGNATURES = {
    "ltn_network_build": [I32, C.POINTER(Gate), I32, I32P, I32, C.POINTER(P)],
    "ltn_netbuf_view": [P, C.POINTER(Network)],
    "ltn_netbuf_data128": [P, C.POINTER(DP)],
    "ltn_netbuf_free": [P],
    "ltn_greedy_path": [C.POINTER(Network), I32P, I32, D, D, U64, I32P],
    "ltn_tree_costs": [C.POINTER(Network), I32P, I32P, I32, C.POINTER(Costs)],
    "ltn_tree_stem": [C.POINTER(Network), I32P, I32P, I32, I32P],
    "ltn_stem_profile": [C.POINTER(Network), I32P, I32P, I32, C.POINTER(StemRow), I32, I32P],
    "ltn_slice_finder": [C.POINTER(Network), I32P, I32, I32P, I32, I32P, I32, I32P],
    "ltn_path_search": [C.POINTER(Network), I32, I32P, I32, C.POINTER(SearchOpts), I32P, I32P, I32,
                        I32P, I32P],
    "ltn_slice_refine": [C.POINTER(Network), I32P, I32, I32P, I32, C.POINTER(RefineOpts), I32P,
                         I32P, C.POINTER(RefineStats)],
    "ltn_slice_greedy_overhead": [C.POINTER(Network), I32P, I32, I32P, I32, I32P, I32, I32P],
    "ltn_tree_reconfigure": [C.POINTER(Network), I32P, I32, I32, I32P, I32, I32, I32P],
    "ltn_plan_load": [C.POINTER(Network), I32P, I32, I32P, C.POINTER(Options), C.POINTER(P)],
    "ltn_plan_describe": [P, C.POINTER(PlanInfo)],
    "ltn_plan_step": [P, I32, C.POINTER(StepInfo)],
    "ltn_workspace_size": [P, I32, I32, C.POINTER(C.c_size_t)],
    "ltn_bind": [P, P, C.c_size_t, I32, P],
    "ltn_execute": [P, U64P, U64, I32, P],
    "ltn_execute_range": [P, U64, U64, I32, P],
    "ltn_execute_scratch": [P, U64P, U64, I32, P, P],
    "ltn_set_params": [P, P],
    "ltn_execute_grad": [P, U64P, U64, I32, P, P, P],
    "ltn_autotune": [P, I32, C.c_char_p],
    "ltn_profile_steps": [P, U64, I32, C.POINTER(C.c_float)],
    "ltn_plan_groups": [P, I32P, I32P, I32P, I32P, I32, I32P],
    "ltn_set_fusion": [P, I32],
    "ltn_set_step_kernel": [P, I32, I32, I32, I32, I32, I32],
    "ltn_step_kernel": [P, I32, I32, I32P, I32P, I32P, I32P],
    "ltn_kernel_name": [I32, I32, I32],
    "ltn_permute": [P, P, I32, I32P, C.c_int64, P],
    "ltn_plan_free": [P],
    "ltn_last_error": [],
    "ltn_version": [],
}
VOID_RET = {"ltn_netbuf_free", "ltn_plan_free"}
STR_RET = {"ltn_last_error", "ltn_version", "ltn_kernel_name"}

_lib = None


def lib():
    """The loaded libltn; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libltn.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_2205_00393_amd.build`")
    h = C.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        f = getattr(h, name)
        f.argtypes = args
        f.restype = None if name in VOID_RET else (C.c_char_p if name in STR_RET else C.c_int32)
    _lib = h
    return h


def check(status):
    if status != LTN_OK:
        raise LtnError(status, lib().ltn_last_error().decode())
    return status


def i32_array(values):
    arr = (C.c_int32 * max(1, len(values)))(*values)
    return arr


def u64_array(values):
    return (C.c_uint64 * max(1, len(values)))(*[int(v) for v in values])


def words_to_int(words):
    return sum(int(w) << (64 * i) for i, w in enumerate(words))
