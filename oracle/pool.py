"""Oracle: classes, refcounts, admission and eviction of the shared block pool
(test infrastructure only).

The paper keeps a function's read-only data on the GPU while it is in use
and for a while after (Sharing-based Memory Management, "Multi-stage
Resource Exit", first stage) and suggests replacing long-inactive functions
when memory is needed ("Other Lessons Learned", third lesson).  It defines no
refcounts, slots or eviction order; the readings fixed here are:

* A class is a set of blocks with identical bytes (see ``oracle.dedup``); a
  resident class occupies one pool slot.  Classes are numbered in creation
  order.  An index maps block content to the resident classes holding it
  (creation order); a registering block joins the first one, or a class
  created earlier in the same registration, and otherwise starts a class.
  An evicted class leaves the index (its functions keep referring to it and
  reload it from their own source); a reloaded class re-enters at the end.
* Registration copies the whole blob and takes no references.  A slot for a
  new class is found by evicting the front zero-reference class not used by
  the registering function so far; if none is left the registration fails,
  its new classes are dropped, and evictions already made stay made.
  At the end of a registration every distinct zero-reference class of the
  function moves to the back of the eviction order, in class order.
* ``setup`` adds one reference to each *distinct* class of the function;
  ``release`` removes them, and classes reaching zero move to the back of the
  eviction order, in class order.  Zero-reference classes stay resident.
* Admission of a setup needs a slot for every non-resident class of the
  function.  Slots come from free budget first, then from evicting front-first
  zero-reference classes the function does not use.  All or nothing: if not
  enough can be freed, the setup fails and nothing changes.  Reloaded classes
  add their length to the bytes copied.
* ``unregister`` (no live setups) drops the function; classes no remaining
  function uses leave the pool.

Pins (tests/test_oracle_pool.py): invariants on random sequences (references
never negative and all zero once every setup is released, a referenced class
is never evicted, resident classes never exceed the budget), equality of the
class partition with ``oracle.dedup`` when nothing is evicted, and
hand-worked sequences.
"""
from __future__ import annotations


class PoolSim:
    def __init__(self, budget_slots: int):
        self.budget = budget_slots
        self.next_class = 0
        self.rc = {}             # class -> references
        self.length = {}         # class -> bytes
        self.content = {}        # class -> content key
        self.resident = set()
        self.index = {}          # content key -> [resident classes, creation/reload order]
        self.lru = []            # zero-reference resident classes, front = next victim
        self.fn_classes = {}     # fn -> class per block
        self.h2d_bytes = 0
        self.live = {}           # setup handle -> fn
        self._next_handle = 1

    # ---------------------------------------------------------------- helpers
    def _distinct(self, fn):
        return sorted(set(self.fn_classes[fn]))

    def _free(self):
        return self.budget - len(self.resident)

    def _evict(self, c):
        self.lru.remove(c)
        self.resident.discard(c)
        chain = self.index[self.content[c]]
        chain.remove(c)
        if not chain:
            del self.index[self.content[c]]

    def _victim(self, protect):
        for c in self.lru:
            if c not in protect:
                return c
        return None

    def _to_back(self, classes):
        for c in sorted(classes):
            if self.rc[c] == 0 and c in self.resident:
                if c in self.lru:
                    self.lru.remove(c)
                self.lru.append(c)

    # ---------------------------------------------------------------- API
    def register(self, fn, keys, lengths) -> bool:
        """``keys[k]`` is a hashable stand-in for block k's bytes (equal keys
        iff equal bytes), ``lengths[k]`` its length."""
        table, created, used = [], [], set()
        for key, L in zip(keys, lengths):
            chain = self.index.get(key)
            if chain:
                c = chain[0]
            else:
                if self._free() <= 0:
                    v = self._victim(used)
                    if v is None:
                        for c in created:      # roll back this registration
                            self.resident.discard(c)
                            self.index.pop(self.content[c], None)
                            for d in (self.rc, self.length, self.content):
                                d.pop(c)
                        return False
                    self._evict(v)
                c = self.next_class
                self.next_class += 1
                self.rc[c], self.length[c], self.content[c] = 0, L, key
                self.resident.add(c)
                self.index[key] = [c]
                created.append(c)
            table.append(c)
            used.add(c)
        self.fn_classes[fn] = table
        self.h2d_bytes += sum(lengths)
        self._to_back(set(table))
        return True

    def setup(self, fn):
        """Returns a handle, or None when admission fails (state unchanged)."""
        distinct = self._distinct(fn)
        missing = [c for c in distinct if c not in self.resident]
        short = len(missing) - self._free()
        if short > 0:
            used = set(distinct)
            victims = [c for c in self.lru if c not in used][:short]
            if len(victims) < short:
                return None
            for v in victims:
                self._evict(v)
        for c in missing:
            self.resident.add(c)
            self.index.setdefault(self.content[c], []).append(c)
            self.h2d_bytes += self.length[c]
        for c in distinct:
            if self.rc[c] == 0 and c in self.lru:
                self.lru.remove(c)
            self.rc[c] += 1
        h = self._next_handle
        self._next_handle += 1
        self.live[h] = fn
        return h

    def release(self, handle):
        fn = self.live.pop(handle)
        zero = []
        for c in self._distinct(fn):
            self.rc[c] -= 1
            assert self.rc[c] >= 0
            if self.rc[c] == 0:
                zero.append(c)
        self._to_back(zero)

    def unregister(self, fn):
        assert fn not in self.live.values()
        mine = set(self.fn_classes.pop(fn))
        still = set()
        for cl in self.fn_classes.values():
            still.update(cl)
        for c in sorted(mine - still):
            if c in self.resident:
                self._evict(c)         # unreferenced, so it is in the order
            self.rc.pop(c)
            self.length.pop(c)
            self.content.pop(c)

    # ---------------------------------------------------------------- views
    def block_state(self, fn):
        """Per block: (class, resident, references)."""
        return [(c, c in self.resident, self.rc[c]) for c in self.fn_classes[fn]]
