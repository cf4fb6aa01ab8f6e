"""Seeded synthetic input generators (data only, no method arithmetic)."""
from .gen import (Response, Workload, config0, config1, config2, scaled,
                  uneven_instance, make_univariate, make_trivariate,
                  random_theta_near)

__all__ = ["Response", "Workload", "config0", "config1", "config2", "scaled",
           "uneven_instance", "make_univariate", "make_trivariate",
           "random_theta_near"]
