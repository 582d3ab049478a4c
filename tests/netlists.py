"""Hand-made netlists for the CPU pins (test helper; no method arithmetic)."""
import numpy as np

FIXED, MACRO = 1, 2


def make(nets, n_inst, flags=None, sizes=None, pos=None, die=(-10, -10, 10, 10),
         offsets=None, ncols=2):
    """Build a netlist dict from a list of nets (lists of instance ids)."""
    net_ptr = np.zeros(len(nets) + 1, np.int32)
    net_ptr[1:] = np.cumsum([len(n) for n in nets])
    pin_node = np.array([v for n in nets for v in n], np.int32)
    if offsets is None:
        offsets = np.zeros((pin_node.size, 2), np.float32)
    if flags is None:
        flags = np.zeros(n_inst, np.uint8)
    if sizes is None:
        sizes = np.ones((n_inst, 2), np.float32)
    if pos is None:
        rng = np.random.default_rng(0)
        pos = rng.uniform(die[0], die[2], (n_inst, ncols))
    return dict(name="hand", n_inst=n_inst, node_flags=np.asarray(flags, np.uint8),
                node_size=np.asarray(sizes, np.float32), net_ptr=net_ptr,
                pin_node=pin_node, pin_off=np.asarray(offsets, np.float32),
                die=np.asarray(die, np.float32), g0=np.asarray(pos, np.float32))


def ring(n):
    """n cells, n two-pin nets i -- i+1 (mod n): the cycle graph C_n."""
    return make([[i, (i + 1) % n] for i in range(n)], n)
