"""Seeded synthetic inputs shared by the library's tests, the oracle and the
benchmark: query DAGs and CNFs.  Holds no decision arithmetic."""
from .query import Query, Expr, NODE_DTYPE  # noqa: F401
from .cnf import CNF, random_ksat, random_3sat_threshold, pigeonhole, concat  # noqa: F401
from .configs import (GenQuery, SAT, UNSAT, config1, config2, config3, config5, oob_2d, oob_1d,  # noqa: F401
                      partition_query)
