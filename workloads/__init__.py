"""Seeded synthetic inputs shared by the library's tests, the oracle and the
benchmark: query DAGs and CNFs.  Holds no decision arithmetic."""
from .query import Query, Expr, NODE_DTYPE  # noqa: F401
from .cnf import (CNF, random_ksat, random_ksat_batch, random_3sat_threshold, pigeonhole,  # noqa: F401
                  concat)
from .generators import (GenQuery, SAT, UNSAT, single_access, batch_1d, batch_2d, random_3sat_sets, random_3sat_train, partition_batch, oob_2d, oob_1d,  # noqa: F401
                      partition_query, oob_lower_1d, batch_lower, batch_wrap)
