"""Parameter continuation (oracle).  Test infrastructure only.

Sec. 3 (the parCont structure) and block PRE.4 of the codes: after redesign
step `loop`, par grows by delta when loop >= istart, par < maxPar and
loop mod isteps == 0.  The codes add delta; a doubling schedule (par times
delta) is also offered because a beta schedule 1, 2, 4, ..., 32 needs it.
"""


def cnt(par, sched, loop):
    """sched = (istart, maxpar, isteps, delta, mode) with mode 'add' | 'mul';
    sched None means no continuation."""
    if sched is None:
        return par
    istart, maxpar, isteps, delta, mode = sched
    if loop >= istart and par < maxpar and loop % isteps == 0:
        return par + delta if mode == "add" else par * delta
    return par
