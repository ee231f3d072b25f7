"""FP64 CPU oracle of iFCTN-TC by PAM -- test infrastructure only (tests,
smoke check, benchmark CPU baseline).  Independent of the HIP library."""
from .ifctn_oracle import *  # noqa: F401,F403
