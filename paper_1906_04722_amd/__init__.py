"""MI355X two-component Shan-Chen throat drainage (hybrid pore-network / LBM
method of Montella, Yuan, Chareyre and Gens).

The compute path is the HIP library built from csrc/ (libsc_lbm.so), reached
through the ctypes binding in `lbm`.
"""
