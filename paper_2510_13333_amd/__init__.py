"""MI355X-native hot path of the NCL method for security-constrained AC-OPF:
assembly, pivot-free supernodal LDL^T and solves of the regularised,
quasi-definite KKT system, behind the C ABI of include/ncl_kkt.h."""
from .ncl import KKT, NclError, load, library_path  # noqa: F401
