"""Seeded synthetic inputs shared by the library's tests, the oracle and the
benchmark: query DAGs and CNFs.  Holds no decision arithmetic."""
from .query import Query, Expr, NODE_DTYPE  # noqa: F401
from .cnf import (CNF, random_ksat, random_ksat_batch, random_3sat_threshold, pigeonhole,  # noqa: F401
                  concat)
from .configs import (GenQuery, SAT, UNSAT, config1, config2, config3, config4, config4_train, config5, oob_2d, oob_1d,  # noqa: F401
                      partition_query, oob_lower_1d, config_lower, config_wrap)
