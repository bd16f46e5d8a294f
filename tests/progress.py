"""Progress lines that reach the terminal while pytest captures test output.

Long GPU tests (full-size oracle runs of several minutes) print a line per step so
that a watcher sees them live; pytest's capture manager is set aside for each line.
"""

import sys

_capman = None


def install(config):
    global _capman
    _capman = config.pluginmanager.getplugin("capturemanager")


def say(*a):
    msg = " ".join(str(v) for v in a)
    if _capman is not None:
        with _capman.global_and_fixture_disabled():
            print(msg, file=sys.stderr, flush=True)
    else:
        print(msg, file=sys.stderr, flush=True)
