"""CPU oracle for RANLUX++ -- test infrastructure only (see ranluxpp.py)."""
from .ranluxpp import *  # noqa: F401,F403
from .ranluxpp import SwbParams, RANLUX  # noqa: F401
